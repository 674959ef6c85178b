// Internal structures shared by the host orchestration (pc_api.cpp) and the
// gfx950 kernels (pc_kernels.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pc {

constexpr int kMaxSpecies = 8;
constexpr int kScanTile = 2048;   // bins per scan tile (256 threads x 8)
constexpr int kScanTileLog2 = 11;
static_assert(kScanTile == 1 << kScanTileLog2, "scan tile is a power of two");
constexpr int kTileReps = 16;      // replicated tile counters for grids of few tiles
constexpr int kTileRepsMaxTiles = 1024;
constexpr int kFixShift = 32;     // deposit fixed point: value * 2^32 in uint64

// Per-instance table (device), 32 bytes.
struct InstInfo {
    uint32_t agent_base;   // first row of the instance in id-ordered arrays
    uint32_t n_agents;
    uint32_t bin_base;     // first global bin of the instance
    uint32_t node_base;    // first global node of the instance
    uint32_t key0, key1;   // Philox key (lo32(seed), hi32(seed) ^ instance)
    float chi_scale;
    uint32_t stream;       // noise stream index (Philox key and counter word 2)
};

// Everything a step kernel needs, passed by value.
struct StepParams {
    int32_t dim, periodic, n_species, n_inst;
    int32_t nb;            // bins per axis
    int32_t stencil;       // 3: (3)^dim bins ; 2: (2)^dim bins picked by half-bin side
    int32_t bin_order;     // 0: row-major, x fastest (the only order built)
    int32_t grid_n;
    int32_t n_total;       // agents over all instances
    int32_t nodes_per_inst;
    int32_t bins_per_inst;
    int32_t has_uptake;
    int32_t deposit_agg;   // 1: LDS-aggregated deposit; 0: direct device atomics
    int32_t sort_rows;     // 1: a lane walks its stencil rows longest first
    float L, halfL;
    float inv_bin;         // nb / L
    float bin_w;           // L / nb in float32 arithmetic
    float h, inv_h, inv_2h, inv_h2;
    float dt, k;
    int32_t tile_totals;   // 1: the histogram also totals each scan tile
    int32_t tile_reps;     // counters per tile total (1 or kTileReps), picked by wave
    float fcap;            // upper clamp of the harmonic force factor, 1e10 k max d
    float cell_top;        // largest lower-corner index as float (n-1 periodic, n-2 walls)
    float cut2[kMaxSpecies * kMaxSpecies];  // float32 squared contact distances
    float dij[kMaxSpecies * kMaxSpecies];   // contact distances
    float amp[kMaxSpecies];                 // sqrt(2 D_s dt)
    float chi[kMaxSpecies];
    float src_fx[kMaxSpecies];              // source_s * 2^32
    float upt_fx[kMaxSpecies];              // uptake_s * 2^32
    int32_t has_react;
    int32_t react_to[kMaxSpecies];          // -1: no switch
    float react_p[kMaxSpecies];             // react_rate dt rounded up to float
    float react_cdt[kMaxSpecies];           // react_rate_c dt
    // Gaussian kernel density deposit (bandwidth eps_s = diameter_s)
    int32_t kde;
    float kde_R;                            // largest truncation radius
    float kde_R2[kMaxSpecies];              // (kde_radius eps_s)^2
    float kde_norm[kMaxSpecies];            // (2 pi eps_s^2)^(-dim/2)
    float kde_l2e[kMaxSpecies];             // log2(e) / (2 eps_s^2)
    float src_f[kMaxSpecies], upt_f[kMaxSpecies];
    // pair interaction: 0 harmonic, 1 exponential, 2 hard spheres (no force;
    // overlaps corrected after the update); tamed Euler pair drift
    int32_t potential, tamed;
    float hs_share[kMaxSpecies * kMaxSpecies];  // 2 D_i / (D_i + D_j)
};

struct PdeParams {
    int32_t dim, periodic, grid_n, nodes_per_inst;
    int64_t n_nodes_total;
    float dts, D_c, gamma, inv_h2;
    float fx_to_density;   // 2^-32 / h^dim
    float inv_hd;          // 1 / h^dim
    int32_t has_uptake;
    int32_t kde;           // 1: sources are kernel-density pairs (sigma, upsilon)
    int32_t kde_clear;     // 1: the last substep clears the pairs (agent-side scatter)
};

// Flag bits latched by kernels in the device flag word.
enum : uint32_t {
    FLAG_NONFINITE = 1u << 0,
    FLAG_BAD_SPECIES = 1u << 1,
    FLAG_INTERNAL = 1u << 2,        // a kernel's own bound check failed (a library bug)
    FLAG_WARN_POSITIVITY = 1u << 8,
    FLAG_WARN_CLAMPED = 1u << 9,
    FLAG_WARN_REACTION = 1u << 10,
};

// Device buffers carved from the caller's workspace.
struct Buffers {
    float4 *P[3];          // positions (x, y, z, bits(inst << 8 | species))
    uint32_t *I[3];        // local ids, same order as P[k]
    uint32_t *count;       // bins_total + 1
    uint32_t *start;       // bins_total + 1
    uint32_t *tile_sum;    // ceil((bins_total + 1) / kScanTile): exclusive tile prefixes
    uint32_t *tile_cnt;    // kTileReps x that: agents per scan tile (tile_reps counters
                           // each), added with the bin counts
    float *c[2];           // chemical, two buffers for substeps
    unsigned long long *S_src, *S_upt;  // fixed-point deposits
    uint32_t *slab_cnt;    // per node slab: its agent count if handed over, else 0
    uint32_t *slab_tab;    // per node slab: the run table of a handed-over slab
    InstInfo *inst;
    uint8_t *species_id;   // species in id order (for set_state)
    uint32_t *step;        // device step counter
    uint32_t *flags;
    // reverse mode (present when the workspace holds a segment)
    float *seg_x;          // (seg_steps + 1) x n_total x dim, id order
    float *seg_c;          // seg_steps x nodes_total
    float *lamX[2];        // n_total x dim
    float4 *lamY;          // n_total, cell-sorted order of the step
    float *lamC[2];        // nodes_total
    float *aSrc, *aUpt;    // dL/dS at nodes
    float *lamG;           // dim x nodes_total
    float *csub;           // n_sub x nodes_total
    double *dth;           // 3 x n_inst
};

struct AdjArgs {
    const float *xnext;    // X^{n+1}, id order, n_total x dim
    const float *lamX_in;  // dL/dX^{n+1}
    const float *aSrc, *aUpt;  // dL/dS at nodes
    float4 *lamY;          // dL/dy (pre-boundary), cell-sorted order (the pair walk's)
    float *lamX_out;       // dL/dX^n (drift and identity terms; pair term added later)
    float *lamG;           // dL/d(node gradient), dim x nodes_total
    double *dth;           // 3 per instance: d/d scale of chi, k, D
    int64_t nodes_total;
    uint32_t step;         // step counter of X^n
};

struct LossArgs {
    int m, dim, n_taps, radius;
    float L, inv_hh;       // histogram spacing L/m and its inverse
    int64_t H;             // m^dim
    float taps[65];
};


// Launch wrappers implemented in pc_kernels.hip.
void launch_init_agents(const StepParams &p, const Buffers &b, const float *x, const uint8_t *sp,
                        int write_species, hipStream_t s);
void launch_bin(const StepParams &p, const Buffers &b, int src, int block, hipStream_t s);
void launch_scan(const StepParams &p, const Buffers &b, int64_t n_bins_total, hipStream_t s);
void launch_scatter(const StepParams &p, const Buffers &b, int src, int dst, int block,
                    hipStream_t s);
void launch_stable(const StepParams &p, const Buffers &b, int src, int dst, int block,
                   hipStream_t s);
void launch_update(const StepParams &p, const Buffers &b, int src, int dst, int cbuf, int block,
                   hipStream_t s);
void launch_deposit(const StepParams &p, const Buffers &b, int src, hipStream_t s);
void launch_pde(const PdeParams &q, const Buffers &b, int cin, int cout, int last,
                hipStream_t s);
void launch_zero_u32(uint32_t *d, int64_t n, hipStream_t s);
void launch_kde(const StepParams &p, const Buffers &b, int src, hipStream_t s);
void launch_overlap(const StepParams &p, const Buffers &b, int src, int dst, int block,
                    hipStream_t s);
size_t chem_inst_lds_bytes(const PdeParams &q);
// owner-computes deposit by slabs of nodes (pc_deposit.hip); with fuse_pde
// also the single PDE substep of the step (and the step counter).  Slabs
// with more than split agents are handed to an agent-parallel pass.
struct SlabShape {
    int By, Bz, nby, nbz;
    int64_t nslabs;        // over all instances
    size_t lds_bytes;      // LDS sums per deposited field
    int assist_blocks;     // grid of k_slab_assist: the work-groups resident at once
};
bool chem_slab_shape(int dim, int n, double bins_per_cell, int n_inst, SlabShape &sh);
// Size the hand-over kernel's grid for the current device: work-groups per
// CU at its LDS use times the CU count (1024 if the runtime cannot say).
void chem_slab_assist_grid(const StepParams &p, SlabShape &sh);
size_t chem_slab_table_words();
// classify 0: the slabs were classified (and the heavy ones handed over)
// by launch_scatter_classify after this step's scan
void launch_chem_slabs(const StepParams &p, const PdeParams &q, const Buffers &b,
                       const SlabShape &sh, uint32_t split, int src, int cur, int fuse_pde,
                       hipStream_t s, int classify = 1);
// The scatter of P[src] into P[dst] by the counts and starts of the scan,
// with the slab classification of launch_chem_slabs in the same grid.
void launch_scatter_classify(const StepParams &p, const PdeParams &q, const Buffers &b,
                             const SlabShape &sh, uint32_t split, int src, int dst,
                             hipStream_t s);
void launch_chem_inst(const StepParams &p, const PdeParams &q, const Buffers &b, int src, int cur,
                      int n_sub, hipStream_t s);
int launch_species_hist(const StepParams &p, const Buffers &b, int src, int m, float s,
                        uint32_t *counts, uint32_t *totals, hipStream_t st);
void launch_field_mean(const float *c, int n_inst, int64_t G, float *out, hipStream_t st);
void launch_positions(const StepParams &p, const Buffers &b, int src, float *out,
                      hipStream_t s);
void launch_species(const StepParams &p, const Buffers &b, int src, uint8_t *out, hipStream_t s);
void launch_apply_species(const StepParams &p, const Buffers &b, int src, const uint8_t *sp,
                          hipStream_t s);
void launch_debug_pairs(const StepParams &p, const Buffers &b, int src, uint32_t *count,
                        unsigned long long *hash, float *F, int block, hipStream_t s);
void launch_pde_ptr(const PdeParams &q, const float *cin, float *cout, unsigned long long *Ssrc,
                    unsigned long long *Supt, int last, uint32_t *flags, hipStream_t s);
void launch_set_u32(uint32_t *ptr, uint32_t v, hipStream_t s);
// reverse mode and loss (pc_adjoint.hip)
void launch_adj_pde(const PdeParams &q, const float *mu_in, float *mu_out, const float *cprev,
                    const Buffers &b, float *aSrc, float *aUpt, int first, int last,
                    hipStream_t s);
void launch_adj_agent(const StepParams &p, const AdjArgs &A, const Buffers &b, int src,
                      const float *c, hipStream_t s);
void launch_adj_pair(const StepParams &p, const Buffers &b, int src, const float4 *lamY,
                     float *lamX_out, hipStream_t s);
void launch_adj_grad(const PdeParams &q, float inv_2h, const float *mu0, const float *lamG,
                     float *lamC_out, hipStream_t s);
void launch_zero_f32(float *d, int64_t n, hipStream_t s);
void launch_zero_f64(double *d, int64_t n, hipStream_t s);
void launch_zero_u64(unsigned long long *d, int64_t n, hipStream_t s);
void launch_loss(const LossArgs &a, const StepParams &p, const Buffers &b, int n_inst,
                 const float *target, unsigned long long *hist, float *buf0, float *buf1,
                 double *loss, float *dLdX, float *rho_out, hipStream_t s);
void launch_copy_f32(float *dst, const float *src, int64_t n, hipStream_t s);

}  // namespace pc
