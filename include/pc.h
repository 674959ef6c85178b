/*
 * pc.h — C ABI of the MI355X (gfx950) library for the hybrid chemotaxis step
 * of Bruna, Maini & Robinson, "Particle-based simulations of
 * reaction-diffusion processes with Aboria" (arXiv:1805.11007).
 *
 * One time step (Sect. 2 and 3 of the paper, in the order of its listings):
 *   1. cell-list binning of the agents (counting sort; Sect. 2.2 and the
 *      neighbour-search set-up of Sect. 3.1);
 *   2. pairwise soft-sphere repulsion F = k (d - r) r_hat for r < d over the
 *      neighbour bins (interaction loop of Sect. 3.2; eqs. sde_alpha/beta);
 *   3. chemotactic drift chi * grad c interpolated multilinearly from the
 *      node grid (Sect. 2.3 and 3.6);
 *   4. Euler-Maruyama update with Philox4x32-10 normals (eq. sde_EM) and the
 *      periodic or reflecting boundary (Sect. 3.2);
 *   5. piecewise-linear deposit of cell source / uptake at the new positions
 *      (Sect. 2.3, eq. random_measure);
 *   6. forward-Euler, centred-difference update of the chemical (eq. pde_c,
 *      Sect. 3.5), in substeps when the explicit limit requires them.
 *
 * Several independent instances (realisations) of one model can be stepped
 * together; each has its own agents, bins, grid and noise key.
 *
 * Conventions for every entry point:
 *   - Return value: PC_OK (0) or a negative PC_E* code; nothing throws.
 *     pc_strerror() names a code; pc_last_error() gives the message of the
 *     last failure on the calling thread.
 *   - Pointers named *_dev are device pointers (HIP device memory on the
 *     device that was current at pc_create).  Pointers without the suffix
 *     are host pointers.
 *   - The caller owns all device memory, including the workspace; the
 *     library never allocates or frees device memory after pc_create.  The
 *     handle itself is a small host object freed by pc_destroy.
 *   - All device work is enqueued asynchronously on the stream given to
 *     pc_create unless stated otherwise.  Kernel-side conditions (non-finite
 *     state, positivity warnings) are latched in device flags and reported
 *     by pc_sync / pc_warnings.
 *   - Agent arrays are "instance-major, id order": instance k occupies rows
 *     [base_k, base_k + N_k), base_k = N_0 + ... + N_{k-1}; within an
 *     instance, row i is the agent with stable id i.
 *   - Grid arrays are instance-major, x fastest: node (ix, iy[, iz]) of
 *     instance k is at k*G + ix + n*(iy + n*iz), G = n^dim.
 */
#ifndef PC_H
#define PC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    PC_OK = 0,
    PC_EINVAL = -1,      /* invalid argument or parameter set            */
    PC_EUNSTABLE = -2,   /* explicit PDE substep count above the limit   */
    PC_ENOSPACE = -3,    /* workspace smaller than pc_workspace_bytes    */
    PC_EHIP = -4,        /* HIP runtime error                            */
    PC_ENONFINITE = -5,  /* NaN or Inf reached the state                 */
    PC_ENOTSUP = -6      /* operation not available for this setup       */
};

/* Warning bits (pc_warnings). */
enum {
    PC_WARN_DT_RULE = 1u,      /* sqrt(2 (D_i + D_j) dt) >= contact distance (Sect. 2.2) */
    PC_WARN_POSITIVITY = 2u,   /* dt' (gamma + uptake density) >= 1 at some node        */
    PC_WARN_CLAMPED = 4u,      /* a position was clamped into the domain                */
    PC_WARN_REACTION = 8u      /* a switching probability rate dt reached 1 (Sect. 2.1
                                  needs rate dt << 1; the switch was then certain)     */
};

#define PC_MAX_SPECIES 8

typedef struct pc_sim pc_sim;

/* Model and numerics shared by all instances. */
typedef struct {
    int32_t dim;            /* 2 or 3                                                   */
    int32_t periodic;       /* 1: torus [0,L)^dim ; 0: reflecting walls [0,L]^dim       */
    double L;               /* box side                                                 */
    int32_t grid_n;         /* chemical nodes per axis (>= 3); periodic spacing L/n,
                               walls spacing L/(n-1) with nodes on both walls           */
    double dt;              /* time step                                                */
    double k_rep;           /* repulsion stiffness k of F = k (d - r) r_hat             */
    double D_c;             /* chemical diffusivity                                     */
    double gamma;           /* chemical decay rate                                      */
    int32_t pde_substeps;   /* 0: smallest count with D_c dt'/h^2 <= 0.9/(2 dim);
                               > 0: used as given, PC_EUNSTABLE above the limit 1/(2 dim) */
    double bin_size;        /* 0: automatic; else the cell-list bin side (>= cutoff)    */
    int32_t deterministic;  /* 1: agents ordered by id inside each bin and every lane
                               walks its stencil rows in a fixed order, so results are
                               bitwise reproducible run to run and an instance of a
                               batch evolves bit for bit as it does alone; 0: the
                               counting sort's atomics order each bin and a lane walks
                               its rows longest first (float summation order only)      */
    int32_t block;          /* 0: 128; else work-group size of the agent kernels
                               (64, 128, 256, 512 or 1024)                              */
    int32_t bin_order;      /* must be 0: row-major bins (x fastest); others PC_ENOTSUP   */
    int32_t deposit_mode;   /* 0: automatic; 1: contributions summed per work-group in
                               LDS before the device atomics; 2: device atomics only;
                               3: deposit and PDE substeps of each instance in one
                               work-group, with the deposit sums in LDS (needs them to
                               fit: 8 bytes x grid_n^dim x (2 with uptake, else 1));
                               4: owner-computes slabs: the step sorts X^{n+1} before
                               the deposit, and one work-group per slab of nodes
                               (whole x rows, a few y rows and z layers) gathers the
                               agents of its cells through that cell list into LDS and
                               stores each node once, with no device atomics; with one
                               PDE substep it also updates its nodes' field (the
                               deposit never reaches HBM).  Rejected (PC_EINVAL) when
                               bins are so much finer than the grid that a slab's bin
                               layers exceed its run table.  Automatic mode picks 3
                               for batches of >= 64 instances whose sums fit, else 4
                               in 3D, else 1 or 2 by agents per node.  The deposit is
                               an integer sum, so every mode gives the same bits        */
    int32_t deposit_kernel; /* 0: particle-in-cell (piecewise-linear weights);
                               1: Gaussian kernel density (Sect. 2.3): at node p,
                               sigma = sum_i source_i K(p - X_i), upsilon likewise,
                               K(x) = (2 pi e^2)^(-dim/2) exp(-|x|^2 / (2 e^2)), e =
                               the agent's diameter, over |p - X_i| < kde_radius e
                               (minimum image on the torus; no image across walls).
                               In 2D, and in deterministic mode, gathered per node
                               over the cell list of X^{n+1} in a fixed order; in 3D
                               otherwise scattered from the agents by float atomics
                               (last bits vary run to run).  deposit_mode is then
                               ignored (3 and 4 are rejected)                          */
    int32_t slab_split;     /* deposit_mode 4 (slabs): a slab whose cells hold more than
                               this many agents (0: 2048) is handed over: its agents are
                               spread in chunks of 1024 over many work-groups, which
                               add their node sums with device atomics, so that a blob
                               collapsed into a few cells does not serialise on one
                               work-group.  The sums are integers: the bits do not
                               depend on it.  Must be >= 0                              */
    double kde_radius;      /* truncation radius in bandwidths (0: 3); kde_radius times
                               the largest diameter must be < L/2                       */
    int32_t potential;      /* pair interaction with contact distance d = mean diameter:
                               0: harmonic soft sphere u = (k_rep/2)(d - r)^2, r < d;
                               1: exponential u = k_rep exp(-r/d) (the soft potential
                                  of Sect. 4), cut at r < pot_range d;
                               2: hard spheres (Sect. 2.2): no force; after the update
                                  every pair closer than d is pushed apart by 2 (d - r),
                                  agent i taking D_i / (D_i + D_j) of it, from the same
                                  positions, then the boundary closure again         */
    int32_t tamed;          /* 1: tamed Euler (eq. sde_ETamed): the pair drift F becomes
                               F / (1 + |F| dt); potentials 0 and 1                     */
    double pot_range;       /* range of potential 1 in contact distances (0: 3)          */
} pc_config;

/* One agent species (the paper's cell type).
 *
 * Type switching (eq. Chemo_reactions, simulated with the fixed-step rule of
 * Sect. 2.1): an agent of this species switches to species react_to during
 * a step with probability min(1, (react_rate + react_rate_c c(X)) dt), where
 * c(X) is the multilinear interpolation of the field at the start of the
 * step at the agent's position at the start of the step.  The draw is word
 * 0 of the agent's Philox block with counter (step, id, stream, 1).  The
 * switch takes effect for the deposit of the same step; drift and noise of
 * the step use the species held at its start.  A species switches only if
 * react_to >= 0 and a rate is > 0, so a zero-filled struct has no reaction. */
typedef struct {
    double diameter;  /* contact distance of a pair = mean of the two diameters */
    double D;         /* diffusion coefficient                                  */
    double chi;       /* chemotactic sensitivity (0: no drift)                  */
    double source;    /* secretion rate k_alpha into the chemical               */
    double uptake;    /* consumption rate k_beta (per unit concentration)       */
    int32_t react_to;     /* species switched to (0..n_species-1, not itself)   */
    int32_t reserved;
    double react_rate;    /* constant switching rate (>= 0)                     */
    double react_rate_c;  /* switching rate per unit concentration (>= 0)       */
} pc_species_t;

/* One independent instance. */
typedef struct {
    int32_t n_agents;  /* >= 1                                                  */
    int32_t stream;    /* noise stream index s of the instance; < 0 means its
                          position in the array.  Philox key (lo32(seed),
                          hi32(seed) ^ s), counter (step, id, s, 0), so an
                          instance run alone with the same seed and stream
                          reproduces its run inside a batch                     */
    uint64_t seed;
    double chi_scale;  /* multiplies every species' chi in this instance        */
} pc_instance;

/* Bytes of device workspace pc_create needs for this setup (host-only, pure).
 * Returns 0 if the parameters are invalid (pc_create reports why). */
size_t pc_workspace_bytes(const pc_config *cfg, const pc_species_t *species, int n_species,
                          const pc_instance *inst, int n_inst);

/* Create a simulation handle: the counterpart of the `Simulation(sample)`
 * constructor of the paper's Python interface (Sect. 4).  There a sample
 * number seeds the realisation's random generators (set-up of Sect. 3.1);
 * here each instance carries the noise key of its realisation, so one
 * handle may hold many realisations.  Creation also builds the cell list
 * over the domain (the neighbour-search set-up of Sect. 3.1) and loads the
 * grid vector c of the chemical (Sect. 3.5).
 *   workspace_dev / workspace_bytes: caller-owned device buffer of at least
 *     pc_workspace_bytes(...) bytes, 256-byte aligned, valid until pc_destroy;
 *   x0_dev: float32, sum(N) x dim, instance-major id order, inside the box;
 *   species0_dev: uint8, sum(N), species index < n_species;
 *   c0_dev: float32, n_inst x grid_n^dim;
 *   hip_stream: hipStream_t the work is enqueued on (NULL = default stream).
 * The inputs are copied into the workspace (asynchronously); they may be
 * released once the stream has passed this call.
 * Errors: PC_EINVAL (dim not 2/3, N < 1, grid_n < 3, diameter <= 0,
 * cutoff >= L/2, fewer than 3 bins per axis, species out of range),
 * PC_EUNSTABLE, PC_ENOSPACE, PC_EHIP. */
int pc_create(const pc_config *cfg, const pc_species_t *species, int n_species,
              const pc_instance *inst, int n_inst, void *workspace_dev, size_t workspace_bytes,
              const float *x0_dev, const uint8_t *species0_dev, const float *c0_dev,
              void *hip_stream, pc_sim **out);

/* Enqueue n_steps time steps (n_steps >= 0): the counterpart of
 * `integrate(time)` of Sect. 4, which advances the simulation by a span of
 * time; integrate(T) is round(T / dt) steps (the Python binding's
 * Sim.integrate).  Each step is the Euler-Maruyama update of eq. sde_EM
 * coupled to the forward-Euler update of eq. pde_c, in the order of the
 * listings of Sect. 3.  With pc_use_graph(sim, 1) the steps are replayed
 * from a captured HIP graph (captured on first use).  Errors: PC_EINVAL
 * (null handle, n_steps < 0), PC_EHIP; kernel-side conditions surface at
 * pc_sync. */
int pc_step(pc_sim *sim, int n_steps);

/* Turn HIP-graph replay of pc_step on (1) or off (0).  Not in the paper (a
 * launch mechanism of this library); results are bit for bit those of
 * eager steps. */
int pc_use_graph(pc_sim *sim, int on);

/* Current positions into out_dev (float32, sum(N) x dim, id order): the
 * counterpart of `get_positions()` of Sect. 4.  The paper wraps the
 * particle positions in a NumPy array without copying; here the positions
 * are written into a caller-owned device buffer (which torch wraps without
 * a host copy), because the library keeps them in cell-sorted order.
 * Stream-ordered.  Errors: PC_EINVAL (null argument), PC_EHIP. */
int pc_positions(pc_sim *sim, float *out_dev);

/* Current chemical field into out_dev (float32, n_inst x grid_n^dim): the
 * grid vector c of the chemical at the nodes (Sect. 3.5), which the paper
 * also hands to Python with a grid-data counterpart of its particle-vector
 * wrapper (Sect. 4).  Stream-ordered device-to-device copy.  Errors:
 * PC_EINVAL (null argument), PC_EHIP. */
int pc_field(pc_sim *sim, float *out_dev);

/* Species of every agent into out_dev (uint8, sum(N), id order): the
 * counterpart of `get_type()` of Sect. 4, the cell type alpha / beta of
 * Sect. 3.1 (a species index here).  Stream-ordered.  Errors: PC_EINVAL
 * (null argument), PC_EHIP. */
int pc_species(pc_sim *sim, uint8_t *out_dev);

/* Checkpoint: positions (as pc_positions), field (as pc_field) and the step
 * counter (host value; steps enqueued so far plus the initial counter).
 * The state of Sect. 3 is the particle set (Sect. 3.1) and the grid vector
 * c (Sect. 3.5); the paper saves finished runs to disk from Python
 * (Sect. 4), and this call is the in-memory form of that.  x_dev or c_dev
 * may be NULL to skip that part.  Stream-ordered.  Errors: PC_EINVAL (null
 * handle), PC_EHIP. */
int pc_get_state(pc_sim *sim, float *x_dev, float *c_dev, uint32_t *step);

/* Restore a checkpoint (the inverse of pc_get_state): positions of the
 * particle set (Sect. 3.1) in id order, the grid vector c (Sect. 3.5) and
 * the step counter; the noise of later steps is that of the restored
 * step counter (Philox is keyed by step, id and instance).  Agents take the
 * species last given to pc_create or pc_set_species (switches made by steps
 * since then are undone); x_dev or c_dev may be NULL to keep that part. */
int pc_set_state(pc_sim *sim, const float *x_dev, const float *c_dev, uint32_t step);

/* Set the species of every agent (uint8, sum(N), id order, each below
 * n_species) and make them the species pc_set_state restores; positions,
 * field and step counter are kept.  Values >= n_species are replaced by 0
 * and reported as PC_EINVAL by the next pc_sync.  Stream-ordered; the
 * caller's array may be reused once the stream has passed this point. */
int pc_set_species(pc_sim *sim, const uint8_t *species_dev);

/* Ensemble statistics of the current state, in the style of the experiment
 * of Sect. 4 (Fig. 1: species densities and the chemical averaged over
 * realisations), every instance of the handle being one realisation.
 *   hist_n      bins per axis on [0, L]; an agent's bin on an axis is
 *               floor(x * float32(hist_n / L)) clamped to [0, hist_n - 1],
 *               formed in float32;
 *   counts_dev  (uint32, n_species x hist_n^dim, x fastest; overwritten):
 *               agents of each species in each bin, summed over instances;
 *   totals_dev  (uint32, n_species; overwritten): agents of each species;
 *   c_mean_dev  (float32, grid_n^dim; NULL to skip): the field averaged
 *               over instances node by node (summed in FP64).
 * Densities normalised as in Fig. 1 are counts / totals.  Stream-ordered;
 * no synchronisation.  Errors: PC_EINVAL for null arrays or
 * n_species * hist_n^dim >= 2^31. */
int pc_ensemble_stats(pc_sim *sim, int hist_n, uint32_t *counts_dev, uint32_t *totals_dev,
                      float *c_mean_dev);

/* Wait for the stream; report PC_ENONFINITE if a non-finite value reached
 * the state since the last call, else PC_OK. */
int pc_sync(pc_sim *sim);

/* Warning bits (PC_WARN_*) seen so far; waits for the stream. */
int pc_warnings(pc_sim *sim, uint32_t *bits);

/* Read-only facts about a handle. */
typedef struct {
    int32_t n_total;        /* sum of agents over instances           */
    int32_t n_inst;
    int32_t bins_per_axis;
    int32_t stencil;        /* 3: 3^dim neighbour bins; 2: 2^dim        */
    int64_t n_bins_total;
    int64_t n_nodes_total;
    int32_t pde_substeps;
    int32_t block;
    double bin_side;
    size_t workspace_bytes;
    int32_t deposit_path;   /* deposit in effect: 1, 2, 3 or 4 as deposit_mode (slabs
                               report 5), 4 for the kernel density; never 0          */
    int32_t reserved;
} pc_info_t;
int pc_info(pc_sim *sim, pc_info_t *info);

/* Measurement: run n_steps steps eagerly with HIP events between the
 * stages of each step and return the mean milliseconds per step of every
 * stage in stage_ms[PC_N_STAGES] (host): bin, scan, scatter, stable order,
 * update, deposit, PDE, hard-sphere overlap correction (a stage that does
 * not run reports 0; a sort run twice in a step, as with the kernel density
 * deposit or hard spheres, adds up).  The fused per-instance deposit + PDE
 * path reports both under the deposit.  Synchronises the stream; advances
 * the state like pc_step. */
enum { PC_STAGE_BIN, PC_STAGE_SCAN, PC_STAGE_SCATTER, PC_STAGE_STABLE, PC_STAGE_UPDATE,
       PC_STAGE_DEPOSIT, PC_STAGE_PDE, PC_STAGE_OVERLAP, PC_N_STAGES };
int pc_profile_steps(pc_sim *sim, int n_steps, double *stage_ms);

/* Release the handle (does not touch caller memory): the end of the
 * `Simulation` object's life (Sect. 4).  Destroys the captured graphs; the
 * caller frees the workspace after the stream has passed the last call.
 * A NULL handle is accepted (PC_OK). */
int pc_destroy(pc_sim *sim);

const char *pc_strerror(int code);
const char *pc_last_error(void);

/* --- test / debug entry points: the step's own kernels with extra output --- */

/* Neighbour sets of the current state, as decided inside the pair kernel:
 * per agent (id order) the number of agents j != i with float32
 * |minimage(x_j - x_i)|^2 < ((d_i + d_j)/2)^2 (rounded to float32) and the
 * wrap-around sum over those j of splitmix64(id_j).  count_dev: uint32,
 * hash_dev: uint64, both sum(N). */
int pc_debug_neighbours(pc_sim *sim, uint32_t *count_dev, uint64_t *hash_dev);

/* Pair forces of the current state (float32, sum(N) x dim, id order), from
 * the update's own walk over the stencil rows (same order of summation). */
int pc_debug_forces(pc_sim *sim, float *F_dev);

/* --- differentiation (reverse mode through the step; not in the paper) ---
 *
 * pc_adjoint_segment: reverse sweep over n_steps steps starting from the
 * current state, with the noise of every step fixed by the Philox keys.
 *   lamX_in_dev  (float32, sum(N) x dim, id order) and lamC_in_dev (float32,
 *                n_inst x G): dL/dX and dL/dc after the n_steps steps;
 *   lamX_out_dev, lamC_out_dev: receive dL/dX and dL/dc of the current state;
 *   dtheta_out   (host, 3 doubles per instance): dL/ds for multiplicative
 *                scales s of every species' chi, of k and of every species'
 *                D, taken at s = 1 (so dL/dk = dtheta[1] / k, etc.).
 * The segment is recomputed forward inside the call (checkpointing); the
 * state is restored to what it was, and the call synchronises the stream.
 * Needs a workspace of pc_workspace_bytes_adjoint(..., seg_steps) bytes with
 * 1 <= n_steps <= seg_steps.  Errors: PC_ENOTSUP without segment storage,
 * when a species has a type switch (a discrete event), or for a setup other
 * than the harmonic potential with the particle-in-cell deposit and no
 * taming; PC_EINVAL for bad arguments, PC_EHIP. */
size_t pc_workspace_bytes_adjoint(const pc_config *cfg, const pc_species_t *species,
                                  int n_species, const pc_instance *inst, int n_inst,
                                  int seg_steps);
int pc_adjoint_segment(pc_sim *sim, const float *lamX_in_dev, const float *lamC_in_dev,
                       int n_steps, float *lamX_out_dev, float *lamC_out_dev,
                       double *dtheta_out);

/* Density-mismatch loss of the current positions, per instance, on a
 * periodic histogram grid of hist_n nodes per axis (spacing L / hist_n):
 * rho = piecewise-linear (cloud-in-cell) histogram divided by the instance's
 * agent count, smoothed by a separable periodic Gaussian of width
 * sigma_bins bins truncated at round(3 sigma_bins) bins (taps normalised
 * to 1), loss_k = sum_l (rho_s,l - target_l)^2.  The paper analyses its
 * runs with histograms of the cell positions; this smooth version is the
 * differentiable one.
 *   target_dev: float32, n_inst x hist_n^dim (x fastest);
 *   work_dev:   caller scratch of pc_density_loss_work_bytes bytes, 256-byte
 *               aligned;
 *   loss_out:   host, n_inst doubles;
 *   dLdX_dev:   NULL or float32 sum(N) x dim, receives dL/dX (id order).
 * Periodic boxes only (PC_ENOTSUP otherwise).  Synchronises the stream. */
size_t pc_density_loss_work_bytes(pc_sim *sim, int hist_n);
int pc_density_loss(pc_sim *sim, const float *target_dev, int hist_n, double sigma_bins,
                    void *work_dev, size_t work_bytes, double *loss_out, float *dLdX_dev);

/* pc_density_loss without a caller buffer, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The histogram, smoothing buffers
 * and per-instance sums live in a file-scope static device array of 4 MiB
 * (one per GPU, held until the process ends), so the call allocates nothing
 * and takes only the inputs and outputs of pc_density_loss:
 *   target_dev, hist_n, sigma_bins, loss_out, dLdX_dev: as pc_density_loss.
 * Limit: pc_density_loss_work_bytes(sim, hist_n) <= 4 MiB, i.e. n_inst *
 * hist_n^dim up to about 262,000 histogram nodes (PC_ENOSPACE beyond).  The
 * array is cleared by kernels at the start of every call.  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (from several
 * host threads or streams) race, so the caller serialises them.  Errors as
 * pc_density_loss, plus PC_EHIP if the array's device address cannot be
 * found.  Synchronises the stream. */
int pc_density_loss_noalloc(pc_sim *sim, const float *target_dev, int hist_n, double sigma_bins,
                            double *loss_out, float *dLdX_dev);

/* The smoothed histogram rho_s of the loss above (float32, n_inst x
 * hist_n^dim) into rho_out_dev, e.g. to build a target from a reference run.
 * Same arguments and errors as pc_density_loss. */
int pc_density_hist(pc_sim *sim, int hist_n, double sigma_bins, void *work_dev,
                    size_t work_bytes, float *rho_out_dev);

#ifdef __cplusplus
}
#endif
#endif /* PC_H */
