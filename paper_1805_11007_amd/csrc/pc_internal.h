// Internal structures shared by the host orchestration (pc_api.cpp) and the
// gfx950 kernels (pc_kernels.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pc {

constexpr int kMaxSpecies = 8;
constexpr int kScanTile = 2048;   // bins per scan tile (256 threads x 8)
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
    int32_t bin_order;     // 0 row-major, 1 bricks of 2^dim bins
    int32_t grid_n;
    int32_t n_total;       // agents over all instances
    int32_t nodes_per_inst;
    int32_t bins_per_inst;
    int32_t has_uptake;
    float L, halfL;
    float inv_bin;         // nb / L
    float h, inv_h, inv_2h, inv_h2;
    float dt, k;
    float cell_top;        // largest lower-corner index as float (n-1 periodic, n-2 walls)
    float cut2[kMaxSpecies * kMaxSpecies];  // float32 squared contact distances
    float dij[kMaxSpecies * kMaxSpecies];   // contact distances
    float amp[kMaxSpecies];                 // sqrt(2 D_s dt)
    float chi[kMaxSpecies];
    float src_fx[kMaxSpecies];              // source_s * 2^32
    float upt_fx[kMaxSpecies];              // uptake_s * 2^32
};

struct PdeParams {
    int32_t dim, periodic, grid_n, nodes_per_inst;
    int64_t n_nodes_total;
    float dts, D_c, gamma, inv_h2;
    float fx_to_density;   // 2^-32 / h^dim
    int32_t has_uptake;
};

// Flag bits latched by kernels in the device flag word.
enum : uint32_t {
    FLAG_NONFINITE = 1u << 0,
    FLAG_BAD_SPECIES = 1u << 1,
    FLAG_WARN_POSITIVITY = 1u << 8,
    FLAG_WARN_CLAMPED = 1u << 9,
};

// Device buffers carved from the caller's workspace.
struct Buffers {
    float4 *P[3];          // positions (x, y, z, bits(inst << 8 | species))
    uint32_t *I[3];        // local ids, same order as P[k]
    uint32_t *bin, *rank;
    uint32_t *count;       // bins_total + 1
    uint32_t *start;       // bins_total + 1
    uint32_t *tile_sum;    // ceil((bins_total + 1) / kScanTile)
    float *c[2];           // chemical, two buffers for substeps
    unsigned long long *S_src, *S_upt;  // fixed-point deposits
    InstInfo *inst;
    uint8_t *species_id;   // species in id order (for set_state)
    uint32_t *step;        // device step counter
    uint32_t *flags;
    // adjoint segment storage (optional)
    float *seg_x;          // seg_steps x n_total x dim, id order
    float *seg_c;          // seg_steps x nodes_total
    float *adj[8];         // adjoint work arrays
    double *adj_red;       // reductions
};

// Launch wrappers implemented in pc_kernels.hip.
void launch_init_agents(const StepParams &p, const Buffers &b, const float *x, const uint8_t *sp,
                        int write_species, hipStream_t s);
void launch_bin(const StepParams &p, const Buffers &b, int src, int block, hipStream_t s);
void launch_scan(const Buffers &b, int64_t n_bins_total, int32_t n_total, hipStream_t s);
void launch_scatter(const StepParams &p, const Buffers &b, int src, int dst, int block,
                    hipStream_t s);
void launch_stable(const StepParams &p, const Buffers &b, int src, int dst, int block,
                   hipStream_t s);
void launch_update(const StepParams &p, const Buffers &b, int src, int dst, int cbuf, int block,
                   hipStream_t s);
void launch_deposit(const StepParams &p, const Buffers &b, int src, hipStream_t s);
void launch_pde(const PdeParams &q, const Buffers &b, int cin, int cout, int last,
                hipStream_t s);
void launch_step_inc(const Buffers &b, hipStream_t s);
void launch_zero_u32(uint32_t *d, int64_t n, hipStream_t s);
void launch_positions(const StepParams &p, const Buffers &b, int src, float *out,
                      hipStream_t s);
void launch_species(const StepParams &p, const Buffers &b, int src, uint8_t *out, hipStream_t s);
void launch_debug_pairs(const StepParams &p, const Buffers &b, int src, uint32_t *count,
                        unsigned long long *hash, float *F, int block, hipStream_t s);
void launch_set_u32(uint32_t *ptr, uint32_t v, hipStream_t s);
void launch_copy_f32(float *dst, const float *src, int64_t n, hipStream_t s);

}  // namespace pc
