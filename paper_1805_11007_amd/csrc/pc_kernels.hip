// gfx950 kernels of one time step of the hybrid chemotaxis model
// (Bruna, Maini & Robinson, arXiv:1805.11007).  Compiled with
// -ffp-contract=off: the neighbour decision r^2 < d^2 must be made in plain
// float32 multiplies and adds, in a fixed order, so that neighbour sets are
// reproducible bit for bit.  Fused multiply-adds are written explicitly
// where they are wanted.
//
// Agent state lives in float4 (x, y, z, bits(instance << 8 | species)) plus
// a uint32 stable id.  A step is: bin -> scan -> scatter (cell-sorted copy)
// [-> stable order by id] -> update (pairs + drift + noise + boundary +
// deposit, writing back into the unsorted buffer in sorted order) -> PDE.
#include <algorithm>

#include "pc_device.h"

namespace pc {

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
__global__ void k_init_agents(StepParams p, const InstInfo *__restrict__ inst,
                              const float *__restrict__ x, const uint8_t *__restrict__ sp,
                              uint8_t *__restrict__ sp_store, int write_species,
                              float4 *__restrict__ P, uint32_t *__restrict__ I,
                              uint32_t *__restrict__ flags) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= p.n_total) return;
    // instance of row g: last k with agent_base <= g
    int lo = 0, hi = p.n_inst - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (inst[mid].agent_base <= (uint32_t)g) lo = mid;
        else hi = mid - 1;
    }
    int s = sp[g];
    if (s >= p.n_species) {
        atomicOr(flags, FLAG_BAD_SPECIES);
        s = 0;
    }
    if (write_species) sp_store[g] = (uint8_t)s;
    float4 v;
    v.x = x[(size_t)g * p.dim + 0];
    v.y = x[(size_t)g * p.dim + 1];
    v.z = p.dim == 3 ? x[(size_t)g * p.dim + 2] : 0.0f;
    v.w = __uint_as_float(((uint32_t)lo << 8) | (uint32_t)s);
    P[g] = v;
    I[g] = (uint32_t)g - inst[lo].agent_base;
}

// Histogram of one agent's bin b: one added to its count and, when the scan
// takes its tile totals from the histogram (totals != 0), to the total of
// b's scan tile.  Neither add returns a value, so the wave does not wait on
// the device atomic (the scatter takes the agent's slot in the bin later,
// when it counts the bin back down to zero), and a run of lanes with one
// bin adds its length with one atomic.  The tile totals are summed
// over the wave first, one device atomic per distinct tile: in the update
// and the overlap pass agents come in cell order and a wave rarely spans
// more than two tiles; after a state load (k_bin, id order) it may span many.
__device__ __forceinline__ void count_bin(uint32_t *__restrict__ count,
                                          uint32_t *__restrict__ tile_cnt, uint32_t b,
                                          int32_t totals, int32_t reps) {
    const WaveRun run = wave_run(b);
    if (run.pos == 0) atomicAdd(count + b, (uint32_t)run.len);
    if (!totals) return;
    // this wave's counter of the tile (reps is 1 or a power of two)
    const uint32_t rep = ((blockIdx.x * blockDim.x + threadIdx.x) >> 6) & (uint32_t)(reps - 1);
    const uint32_t t = b >> kScanTileLog2;
    while (true) {
        const uint32_t lead = __builtin_amdgcn_readfirstlane(t);
        const unsigned long long m = __ballot(t == lead);
        if (t == lead) {
            if (__lane_id() == __builtin_ctzll(m))
                atomicAdd(tile_cnt + (size_t)lead * reps + rep, (uint32_t)__popcll(m));
            break;
        }
    }
}

template <int DIM>
__global__ void k_bin(StepParams p, const InstInfo *__restrict__ inst,
                      const float4 *__restrict__ P, uint32_t *__restrict__ count,
                      uint32_t *__restrict__ tile_cnt) {
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int i = blk * blockDim.x + threadIdx.x;
    if (i >= p.n_total) return;
    const float4 x = P[i];
    const uint32_t b = inst[inst_of(x.w)].bin_base + agent_bin<DIM>(p, x);
    count_bin(count, tile_cnt, b, p.tile_totals, p.tile_reps);
}

// Block-wide exclusive scan of one value per thread (blockDim = 256).
__device__ __forceinline__ uint32_t block_exscan256(uint32_t v, uint32_t *lds, uint32_t &total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) lds[wv] = x;
    __syncthreads();
    uint32_t base = 0;
    for (int k = 0; k < wv; ++k) base += lds[k];
    total = lds[0] + lds[1] + lds[2] + lds[3];
    __syncthreads();
    return base + x - v;
}

// 8 consecutive counts starting at base (a multiple of 8): two 16-byte
// loads when the whole group is in range.
__device__ __forceinline__ void load8(const uint32_t *__restrict__ a, int64_t base, int64_t n,
                                      uint32_t v[8]) {
    if (base + 8 <= n) {
        const uint4 *p4 = reinterpret_cast<const uint4 *>(a + base);
        const uint4 x = p4[0], y = p4[1];
        v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
        v[4] = y.x; v[5] = y.y; v[6] = y.z; v[7] = y.w;
    } else {
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = base + k < n ? a[base + k] : 0u;
    }
}

// Totals of the bin counts of each scan tile, for histograms that did not
// gather them (few bins per agent).
__global__ void __launch_bounds__(256) k_tile_sums(const uint32_t *__restrict__ count,
                                                   int64_t n, uint32_t *__restrict__ tile_cnt) {
    __shared__ uint32_t lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
    uint32_t v[8];
    load8(count, base, n, v);
    const uint32_t s = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    uint32_t tot;
    block_exscan256(s, lds, tot);
    if (threadIdx.x == 0) tile_cnt[blockIdx.x] = tot;
}

// Exclusive scan of the T tile totals (gathered by the histogram or by
// k_tile_sums) into tile_sum by one work-group of 1024 threads: passes of
// 8192 totals, 8 consecutive totals per thread (two 16-byte loads and
// stores), carrying the running total between passes.  With reps counters
// per tile (kTileReps, grids of at most kTileRepsMaxTiles tiles) a tile's
// total is the sum of its counters.  The counters are cleared for the next
// histogram.
__global__ void __launch_bounds__(1024) k_scan_tiles(uint32_t *__restrict__ tile_cnt,
                                                     uint32_t *__restrict__ tile_sum, int T,
                                                     int reps) {
    __shared__ uint32_t lds[16];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t carry = 0;
    for (int64_t off = 0; off < T; off += 8192) {
        const int64_t b0 = off + threadIdx.x * 8;
        uint32_t v[8];
        if (reps == 1) {
            load8(tile_cnt, b0, T, v);
        } else {
            // kTileReps counters per tile, four 16-byte loads, then cleared
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                v[k] = 0u;
                if (b0 + k < T) {
                    uint4 *q = reinterpret_cast<uint4 *>(tile_cnt + (b0 + k) * kTileReps);
#pragma unroll
                    for (int r = 0; r < kTileReps / 4; ++r) {
                        const uint4 u = q[r];
                        v[k] += (u.x + u.y) + (u.z + u.w);
                        q[r] = make_uint4(0u, 0u, 0u, 0u);
                    }
                }
            }
        }
        const uint32_t s = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
        uint32_t x = s;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (lane == 63) lds[wv] = x;
        __syncthreads();
        uint32_t base = carry, total = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t t = lds[k];
            if (k < wv) base += t;
            total += t;
        }
        uint32_t run = base + x - s;
        uint32_t o[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            o[k] = run;
            run += v[k];
        }
        if (b0 + 8 <= T) {
            uint4 *p4 = reinterpret_cast<uint4 *>(tile_sum + b0);
            p4[0] = make_uint4(o[0], o[1], o[2], o[3]);
            p4[1] = make_uint4(o[4], o[5], o[6], o[7]);
            if (reps == 1) {
                uint4 *z4 = reinterpret_cast<uint4 *>(tile_cnt + b0);
                z4[0] = make_uint4(0u, 0u, 0u, 0u);
                z4[1] = make_uint4(0u, 0u, 0u, 0u);
            }
        } else {
            for (int k = 0; k < 8; ++k)
                if (b0 + k < T) {
                    tile_sum[b0 + k] = o[k];
                    if (reps == 1) tile_cnt[b0 + k] = 0u;
                }
        }
        carry += total;
        __syncthreads();
    }
}

// Bin starts of one tile from its counts and the tile's prefix.  A tile
// holding no agent (its prefix equals the next one; the last tile ends at
// n_agents) has only zero counts: its starts are all the prefix, written
// without reading the counts.  The counts stay: the scatter counts them
// back down to zero.
__global__ void __launch_bounds__(256) k_scan_apply(const uint32_t *__restrict__ count, int64_t n,
                                                    const uint32_t *__restrict__ tile_sum,
                                                    uint32_t *__restrict__ start, int T,
                                                    uint32_t n_agents) {
    __shared__ uint32_t lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
    const uint32_t pre = tile_sum[blockIdx.x];
    const uint32_t nxt = (int)blockIdx.x + 1 < T ? tile_sum[blockIdx.x + 1] : n_agents;
    if (pre == nxt) {
        if (base + 8 <= n) {
            uint4 *st4 = reinterpret_cast<uint4 *>(start + base);
            st4[0] = st4[1] = make_uint4(pre, pre, pre, pre);
        } else {
            for (int k = 0; k < 8; ++k)
                if (base + k < n) start[base + k] = pre;
        }
        return;
    }
    uint32_t v[8];
    load8(count, base, n, v);
    const uint32_t s = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7]));
    uint32_t tot;
    uint32_t run = block_exscan256(s, lds, tot) + pre;
    uint32_t o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        o[k] = run;
        run += v[k];
    }
    if (base + 8 <= n) {
        uint4 *st4 = reinterpret_cast<uint4 *>(start + base);
        st4[0] = make_uint4(o[0], o[1], o[2], o[3]);
        st4[1] = make_uint4(o[4], o[5], o[6], o[7]);
    } else {
        for (int k = 0; k < 8; ++k)
            if (base + k < n) start[base + k] = o[k];
    }
}

// Each agent takes a slot in its bin by counting the bin down: the slots
// 0 .. n_b - 1 go to its n_b agents in the order their decrements arrive
// (deterministic mode then orders each bin by id), and the counts are back
// at zero for the next histogram.  A run of lanes with one bin takes its
// slots with one atomic, its first lane's, and shares the old count.
template <int DIM>
__global__ void k_scatter(StepParams p, const float4 *__restrict__ P,
                          const uint32_t *__restrict__ I, uint32_t *__restrict__ count,
                          const uint32_t *__restrict__ start, float4 *__restrict__ Ps,
                          uint32_t *__restrict__ Is) {
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int i = blk * blockDim.x + threadIdx.x;
    if (i >= p.n_total) return;
    scatter_agent<DIM>(p, P, I, count, start, Ps, Is, i);
}

// Deterministic order inside each bin: an agent's slot is its bin start
// plus the number of agents of the bin with a smaller id.
template <int DIM>
__global__ void k_stable(StepParams p, const InstInfo *__restrict__ inst,
                         const float4 *__restrict__ Ps, const uint32_t *__restrict__ Is,
                         const uint32_t *__restrict__ start, float4 *__restrict__ Pd,
                         uint32_t *__restrict__ Id) {
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int j = blk * blockDim.x + threadIdx.x;
    if (j >= p.n_total) return;
    const float4 x = Ps[j];
    const uint32_t b = inst[inst_of(x.w)].bin_base + agent_bin<DIM>(p, x);
    const uint32_t a = start[b], e = start[b + 1], id = Is[j];
    uint32_t r = 0;
    for (uint32_t t = a; t < e; ++t) r += Is[t] < id ? 1u : 0u;
    Pd[a + r] = x;
    Id[a + r] = id;
}

// The fused particle update of one step, one thread per cell-sorted agent:
// pair repulsion at X^n, chemotactic drift from c^n at X^n, Euler-Maruyama
// with Philox normals, boundary closure; then the cell-list bin of X^{n+1},
// counted into the histogram of the next step's counting sort.
// POT: 0 harmonic, 1 exponential, 2 hard spheres (no pair force here).
template <int DIM, int NS, int STENCIL, int POT>
__global__ void __launch_bounds__(1024)
k_update(StepParams p, const InstInfo *__restrict__ inst, const float4 *__restrict__ Ps,
         const uint32_t *__restrict__ Is, const uint32_t *__restrict__ start,
         const float *__restrict__ c, float4 *__restrict__ Pout, uint32_t *__restrict__ Iout,
         uint32_t *__restrict__ count,
         uint32_t *__restrict__ tile_cnt,
         const uint32_t *__restrict__ stepc, uint32_t *__restrict__ flags) {
    __shared__ SpTab tab;
    if (NS == 0) {
        load_tab(p, tab);
        __syncthreads();
    }
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int i = blk * blockDim.x + threadIdx.x;
    if (i >= p.n_total) return;
    const float4 pi = Ps[i];
    const uint32_t id = Is[i];
    const int si = species_of(pi.w);
    // instance tables are equal-sized: the bin and node bases follow from
    // the instance index without waiting for its table entry (whose noise
    // key and chi scale are needed only after the pair loop)
    const uint32_t kin = inst_of(pi.w);
    const uint32_t bin_base = kin * (uint32_t)p.bins_per_inst;
    const uint32_t node_base = kin * (uint32_t)p.nodes_per_inst;
    const InstInfo ii = inst[kin];

    // the row table of the longest-row-first pair walk (a word per stencil
    // row and thread, launched with that much dynamic LDS)
    extern __shared__ uint32_t upd_rows[];
    uint32_t *rowa = STENCIL == 3 ? upd_rows + threadIdx.x : nullptr;
    float F[3] = {0.f, 0.f, 0.f};
    if (POT == 0) {
        ForceVisitor fv{p.k, p.fcap, {0.f, 0.f, 0.f}};
        pair_loop<DIM, NS, STENCIL>(p, tab, Ps, start, bin_base, pi, si, fv, rowa);
        F[0] = fv.F[0];
        F[1] = fv.F[1];
        F[2] = fv.F[2];
    } else if (POT == 1) {
        ExpVisitor ev{p.k, {0.f, 0.f, 0.f}};
        pair_loop<DIM, NS, STENCIL>(p, tab, Ps, start, bin_base, pi, si, ev, rowa);
        F[0] = ev.F[0];
        F[1] = ev.F[1];
        F[2] = ev.F[2];
    }
    if (POT != 2 && p.tamed) {
        // tamed Euler (eq. sde_ETamed): the pair drift becomes F / (1 + |F| dt)
        const float s = 1.0f / (1.0f + sqrtf(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]) * p.dt);
        F[0] *= s;
        F[1] *= s;
        F[2] *= s;
    }

    float drift[3] = {0.f, 0.f, 0.f};
    const float chi = sel<NS>(p.chi, tab.chi, si) * ii.chi_scale;
    if (chi != 0.0f) {
        float g[3];
        grad_interp<DIM>(p, c + node_base, pi, g);
        drift[0] = chi * g[0];
        drift[1] = chi * g[1];
        drift[2] = chi * g[2];
    }

    const U4 w = philox4x32_10(*stepc, id, ii.stream, 0u, ii.key0, ii.key1);
    float xi[3];
    normals<DIM>(w, xi);
    const float amp = sel<NS>(p.amp, tab.amp, si);
    uint32_t flag = 0;
    float4 xn;
    // the increment is summed first and added to the position once, so the
    // new position carries a single rounding at its own scale
    xn.x = boundary(p, pi.x + (p.dt * (F[0] + drift[0]) + amp * xi[0]), flag);
    xn.y = boundary(p, pi.y + (p.dt * (F[1] + drift[1]) + amp * xi[1]), flag);
    xn.z = DIM == 3 ? boundary(p, pi.z + (p.dt * (F[2] + drift[2]) + amp * xi[2]), flag) : 0.0f;
    xn.w = pi.w;
    if (p.has_react) {
        // type switch (eq. Chemo_reactions, fixed-step rule): one more Philox
        // block on counter word 3 = 1; the rate reads c^n at X^n
        const int to = NS == 1 ? p.react_to[0] : (NS == 2 ? (si ? p.react_to[1] : p.react_to[0])
                                                           : p.react_to[si]);
        if (to >= 0) {
            float prob = sel<NS>(p.react_p, p.react_p, si);
            const float rc = sel<NS>(p.react_cdt, p.react_cdt, si);
            if (rc != 0.0f) prob = fmaf(rc, value_interp<DIM>(p, c + node_base, pi), prob);
            const U4 wr = philox4x32_10(*stepc, id, ii.stream, 1u, ii.key0, ii.key1);
            if (uniform24(wr.v[0]) < prob)
                xn.w = __uint_as_float((__float_as_uint(pi.w) & ~0xffu) | (uint32_t)to);
            if (prob >= 1.0f) flag |= FLAG_WARN_REACTION;
        }
    }
    if (!(isfinite(xn.x) && isfinite(xn.y) && isfinite(xn.z))) flag |= FLAG_NONFINITE;
    Pout[i] = xn;
    Iout[i] = id;
    const uint32_t b = bin_base + agent_bin<DIM>(p, xn);
    count_bin(count, tile_cnt, b, p.tile_totals, p.tile_reps);
    if (flag) atomicOr(flags, flag);
}

// Piecewise-linear deposit (fixed point, 2^-32 units) of every agent at its
// new position, one thread per agent.  The 2^dim corner contributions of a
// work-group's agents (contiguous in cell-sorted order, hence spatially
// close) are first summed in an LDS hash table keyed by node, then flushed
// with one device atomic per distinct node.  Integer sums make the result
// independent of the summation order.
constexpr int kDepSlots = 4096;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;

__device__ __forceinline__ void lds_insert(uint32_t *keys, unsigned long long *vs,
                                           unsigned long long *vu, bool upt, uint32_t key,
                                           unsigned long long a, unsigned long long b,
                                           unsigned long long *Ssrc,
                                           unsigned long long *Supt) {
    uint32_t h = (key * 2654435761u) >> 20;  // 12 bits: kDepSlots = 4096
    for (int probe = 0; probe < 16; ++probe) {
        // a plain read finds a node already in the table (the rule in dense
        // regions); only a free slot takes the compare-and-swap
        uint32_t old = __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (old == kEmpty) old = atomicCAS(&keys[h], kEmpty, key);
        if (old == kEmpty || old == key) {
            if (a) atomicAdd(&vs[h], a);
            if (upt && b) atomicAdd(&vu[h], b);
            return;
        }
        h = (h + 1) & (kDepSlots - 1);
    }
    if (a) atomicAdd(Ssrc + key, a);
    if (upt && b) atomicAdd(Supt + key, b);
}

// Corner nodes (instance-local index + base) and fixed-point contributions
// of one agent's piecewise-linear deposit.  Returns false for an agent of a
// species with neither source nor uptake (all contributions zero).
template <int DIM, int NS, bool UPT>
__device__ __forceinline__ bool deposit_corners(const StepParams &p, const SpTab &tab, float4 x,
                                                uint32_t base, uint32_t key[1 << DIM],
                                                unsigned long long cs[1 << DIM],
                                                unsigned long long cu[1 << DIM]) {
    const int s = species_of(x.w);
    const float qs = sel<NS>(p.src_fx, tab.src, s);
    const float qu = UPT ? sel<NS>(p.upt_fx, tab.upt, s) : 0.0f;
    const bool valid = qs != 0.0f || qu != 0.0f;
    Cell cc[3];
    cc[0] = cell_of(p, x.x);
    cc[1] = cell_of(p, x.y);
    if (DIM == 3) cc[2] = cell_of(p, x.z);
    const int n = p.grid_n;
#pragma unroll
    for (int m = 0; m < (1 << DIM); ++m) {
        float ws = qs, wu = qu;
        uint32_t idx = 0, stride = 1;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int up = (m >> a) & 1;
            const float f = up ? cc[a].t : 1.0f - cc[a].t;
            ws *= f;
            if (UPT) wu *= f;
            idx += (uint32_t)(up ? cc[a].i1 : cc[a].i0) * stride;
            stride *= (uint32_t)n;
        }
        key[m] = base + idx;
        cs[m] = valid ? (unsigned long long)__float2ull_rn(ws) : 0ull;
        cu[m] = valid && UPT ? (unsigned long long)__float2ull_rn(wu) : 0ull;
    }
    return valid;
}

// AGG = false skips the LDS table (each contribution goes straight to a
// device atomic): cheaper when agents are sparse next to the nodes, so that
// a work-group's agents rarely share a node.
template <int DIM, int NS, bool UPT, bool AGG>
__global__ void __launch_bounds__(1024)
k_deposit(StepParams p, const InstInfo *__restrict__ inst, const float4 *__restrict__ P,
          unsigned long long *__restrict__ Ssrc, unsigned long long *__restrict__ Supt) {
    constexpr int slots = AGG ? kDepSlots : 1;
    __shared__ uint32_t keys[slots];
    __shared__ unsigned long long vs[slots];
    __shared__ unsigned long long vu[UPT && AGG ? kDepSlots : 1];
    __shared__ SpTab tab;
    if (AGG) {
        for (int q = threadIdx.x; q < kDepSlots; q += blockDim.x) {
            keys[q] = kEmpty;
            vs[q] = 0ull;
            if (UPT) vu[q] = 0ull;
        }
    }
    if (NS == 0) load_tab(p, tab);
    __syncthreads();
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int i = blk * blockDim.x + threadIdx.x;
    // corner keys and fixed-point contributions (zero for idle lanes)
    uint32_t key[1 << DIM];
    unsigned long long cs[1 << DIM], cu[1 << DIM];
    bool valid = false;
    if (i < p.n_total) {
        const float4 x = P[i];
        valid = deposit_corners<DIM, NS, UPT>(p, tab, x, inst[inst_of(x.w)].node_base, key, cs,
                                              cu);
    } else {
#pragma unroll
        for (int m = 0; m < (1 << DIM); ++m) {
            key[m] = kEmpty;
            cs[m] = cu[m] = 0ull;
        }
    }
    auto emit = [&](uint32_t k, unsigned long long a, unsigned long long b) {
        if (AGG) {
            lds_insert(keys, vs, vu, UPT, k, a, b, Ssrc, Supt);
        } else {
            if (a) atomicAdd(Ssrc + k, a);
            if (UPT && b) atomicAdd(Supt + k, b);
        }
    };
    // In dense clusters every lane of the wave often deposits into the same
    // 2^dim nodes: sum over the wave first and insert once per node.
    const uint32_t k0 = valid ? key[0] : kEmpty;
    const uint32_t f0 = __builtin_amdgcn_readfirstlane(k0);
    const bool uniform = f0 != kEmpty && __all(!valid || k0 == f0);
    if (uniform) {
#pragma unroll
        for (int m = 0; m < (1 << DIM); ++m) {
            unsigned long long a = cs[m], b = cu[m];
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) {
                a += __shfl_xor(a, d, 64);
                if (UPT) b += __shfl_xor(b, d, 64);
            }
            if ((threadIdx.x & 63) == 0) emit(key[m], a, b);
        }
    } else if (valid) {
#pragma unroll
        for (int m = 0; m < (1 << DIM); ++m)
            if (cs[m] || cu[m]) emit(key[m], cs[m], cu[m]);
    }
    if (!AGG) return;
    __syncthreads();
    for (int q = threadIdx.x; q < kDepSlots; q += blockDim.x) {
        const uint32_t k = keys[q];
        if (k == kEmpty) continue;
        if (vs[q]) atomicAdd(Ssrc + k, vs[q]);
        if (UPT && vu[q]) atomicAdd(Supt + k, vu[q]);
    }
}

// Deposit and every PDE substep of one instance in one work-group, for
// batches of many small instances: the instance's deposit sums stay in LDS
// (never in HBM) and the field is read and written once per substep.  The
// agents of instance k occupy rows [agent_base, agent_base + n_agents) of
// the state in every order the step uses (instance-major bins).  The same
// corner contributions and node update as k_deposit + k_pde, so the same
// bits.  Substeps ping-pong between the two field buffers, starting from
// buffer `cur`; the barrier between substeps orders them.
template <int DIM, int NS, bool UPT>
__global__ void __launch_bounds__(1024)
k_chem_inst(StepParams p, PdeParams q, const InstInfo *__restrict__ inst,
            const float4 *__restrict__ P, float *__restrict__ c0, float *__restrict__ c1, int cur,
            int n_sub, uint32_t *__restrict__ flags, uint32_t *__restrict__ stepc) {
    // the last kernel of a step advances the step counter (the update,
    // which reads it, has finished)
    if (blockIdx.x == 0 && threadIdx.x == 0) *stepc += 1u;
    extern __shared__ unsigned long long S[];  // G source sums, then G uptake sums
    __shared__ SpTab tab;
    const int G = q.nodes_per_inst;
    for (int l = threadIdx.x; l < G * (UPT ? 2 : 1); l += blockDim.x) S[l] = 0ull;
    if (NS == 0) load_tab(p, tab);
    __syncthreads();
    const InstInfo ii = inst[blockIdx.x];
    for (uint32_t i = threadIdx.x; i < ii.n_agents; i += blockDim.x) {
        uint32_t key[1 << DIM];
        unsigned long long cs[1 << DIM], cu[1 << DIM];
        if (!deposit_corners<DIM, NS, UPT>(p, tab, P[ii.agent_base + i], 0u, key, cs, cu))
            continue;
#pragma unroll
        for (int m = 0; m < (1 << DIM); ++m) {
            if (cs[m]) atomicAdd(&S[key[m]], cs[m]);
            if (UPT && cu[m]) atomicAdd(&S[G + key[m]], cu[m]);
        }
    }
    __syncthreads();
    const int n = q.grid_n;
    uint32_t flag = 0;
    for (int m = 0; m < n_sub; ++m) {
        const float *src = (((cur + m) & 1) ? c1 : c0) + ii.node_base;
        float *dst = (((cur + m + 1) & 1) ? c1 : c0) + ii.node_base;
        for (int l = threadIdx.x; l < G; l += blockDim.x) {
            const int ic[3] = {l % n, (l / n) % n, DIM == 3 ? l / (n * n) : 0};
            dst[l] = pde_node<DIM>(q, src, ic, S[l], UPT ? S[G + l] : 0ull, flag);
        }
        if (m + 1 < n_sub) __syncthreads();
    }
    if (flag) atomicOr(flags, flag);
}

// PDE substep, one thread per node; the last substep of a step clears the
// deposits for the next step.
// KDE: the source array holds (sigma, upsilon) float pairs.  The per-node
// gather rewrites every pair each step; the agent-side scatter adds into
// them, so with it (q.kde_clear) the last substep clears the pairs it read.
// stepc (non-null on the last substep of a step): the step counter,
// advanced by node 0.
// One work-group per grid row along x: the instance and the (y, z) of the
// row are wave-uniform, so no thread divides by the grid size.
template <int DIM, bool KDE>
__global__ void __launch_bounds__(256)
k_pde(PdeParams q, const float *__restrict__ cin, float *__restrict__ cout,
      unsigned long long *__restrict__ Ssrc, unsigned long long *__restrict__ Supt, int last,
      uint32_t *__restrict__ flags, uint32_t *__restrict__ stepc) {
    const uint32_t row = blockIdx.x;
    if (stepc && row == 0 && threadIdx.x == 0) *stepc += 1u;
    const int n = q.grid_n;
    const uint32_t rows_per_inst = DIM == 3 ? (uint32_t)n * (uint32_t)n : (uint32_t)n;
    const uint32_t k = row / rows_per_inst;
    const uint32_t rr = row - k * rows_per_inst;
    const int iy = (int)(rr % (uint32_t)n), iz = DIM == 3 ? (int)(rr / (uint32_t)n) : 0;
    const float *cb = cin + (int64_t)k * q.nodes_per_inst;
    uint32_t flag = 0;
    for (int ix = threadIdx.x; ix < n; ix += blockDim.x) {
        const int64_t l = (int64_t)row * n + ix;
        const int ic[3] = {ix, iy, iz};
        if (KDE) {
            float2 *dens = reinterpret_cast<float2 *>(Ssrc);
            const float2 su = dens[l];
            cout[l] = pde_node_dens<DIM>(q, cb, ic, su.x, su.y, flag);
            if (last && q.kde_clear && (su.x != 0.0f || su.y != 0.0f))
                dens[l] = make_float2(0.0f, 0.0f);
            continue;
        }
        const unsigned long long sS = Ssrc[l], sU = q.has_uptake ? Supt[l] : 0ull;
        cout[l] = pde_node<DIM>(q, cb, ic, sS, sU, flag);
        if (last) {
            if (sS) Ssrc[l] = 0ull;
            if (sU) Supt[l] = 0ull;
        }
    }
    if (flag) atomicOr(flags, flag);
}

__global__ void k_zero_u32(uint32_t *__restrict__ d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = 0u;
}

__global__ void k_positions(StepParams p, const InstInfo *__restrict__ inst,
                            const float4 *__restrict__ P, const uint32_t *__restrict__ I,
                            float *__restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p.n_total) return;
    const float4 x = P[j];
    const size_t row = inst[inst_of(x.w)].agent_base + I[j];
    out[row * p.dim + 0] = x.x;
    out[row * p.dim + 1] = x.y;
    if (p.dim == 3) out[row * p.dim + 2] = x.z;
}

__global__ void k_species(StepParams p, const InstInfo *__restrict__ inst,
                          const float4 *__restrict__ P, const uint32_t *__restrict__ I,
                          uint8_t *__restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p.n_total) return;
    const float4 x = P[j];
    out[inst[inst_of(x.w)].agent_base + I[j]] = (uint8_t)species_of(x.w);
}

// Species of every agent from an id-ordered array (pc_set_species).
__global__ void k_apply_species(StepParams p, const InstInfo *__restrict__ inst,
                                float4 *__restrict__ P, const uint32_t *__restrict__ I,
                                const uint8_t *__restrict__ sp, uint32_t *__restrict__ flags) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p.n_total) return;
    const float4 x = P[j];
    const uint32_t k = inst_of(x.w);
    uint32_t s = sp[inst[k].agent_base + I[j]];
    if (s >= (uint32_t)p.n_species) {
        atomicOr(flags, FLAG_BAD_SPECIES);
        s = 0;
    }
    P[j].w = __uint_as_float((k << 8) | s);
}

template <int DIM, int NS, int STENCIL, int POT>
__global__ void __launch_bounds__(1024)
k_debug_pairs(StepParams p, const InstInfo *__restrict__ inst, const float4 *__restrict__ Ps,
              const uint32_t *__restrict__ Is, const uint32_t *__restrict__ start,
              uint32_t *__restrict__ count, unsigned long long *__restrict__ hash,
              float *__restrict__ Fo) {
    __shared__ SpTab tab;
    if (NS == 0) {
        load_tab(p, tab);
        __syncthreads();
    }
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.n_total) return;
    const float4 pi = Ps[i];
    const int si = species_of(pi.w);
    const InstInfo ii = inst[inst_of(pi.w)];
    const size_t row = ii.agent_base + Is[i];
    // the update's walk, with its LDS row table (same launch shape, so the
    // same waves and the same row order)
    extern __shared__ uint32_t dbg_rows[];
    uint32_t *rowa = STENCIL == 3 ? dbg_rows + threadIdx.x : nullptr;
    uint32_t cnt;
    unsigned long long hs;
    float F[3];
    if (POT == 1) {
        DebugVisitor<ExpVisitor> dv{ExpVisitor{p.k, {0.f, 0.f, 0.f}}, (uint32_t)i, Is, 0u, 0ull};
        pair_loop<DIM, NS, STENCIL>(p, tab, Ps, start, ii.bin_base, pi, si, dv, rowa);
        cnt = dv.cnt;
        hs = dv.hs;
        F[0] = dv.fv.F[0], F[1] = dv.fv.F[1], F[2] = dv.fv.F[2];
    } else {
        // hard spheres exert no force; with k = 0 the factor is 0 * inf at r = 0
        const float k = POT == 0 ? p.k : 0.0f;
        DebugVisitor<ForceVisitor> dv{ForceVisitor{k, p.fcap, {0.f, 0.f, 0.f}}, (uint32_t)i, Is,
                                      0u, 0ull};
        pair_loop<DIM, NS, STENCIL>(p, tab, Ps, start, ii.bin_base, pi, si, dv, rowa);
        cnt = dv.cnt;
        hs = dv.hs;
        const bool force = k != 0.0f;
        F[0] = force ? dv.fv.F[0] : 0.0f;
        F[1] = force ? dv.fv.F[1] : 0.0f;
        F[2] = force ? dv.fv.F[2] : 0.0f;
    }
    if (count) count[row] = cnt;
    if (hash) hash[row] = hs;
    if (Fo)
        for (int a = 0; a < DIM; ++a) Fo[row * DIM + a] = F[a];
}

// Hard-sphere overlap correction (Sect. 2.2) at the updated, cell-sorted
// positions: every pair closer than its contact distance pushes i away by
// 2 (d - r) D_i / (D_i + D_j); all pushes come from the same positions.
// Then the boundary closure, and the bin of the corrected position counted
// for the counting sort of the next step, as the update kernel does.
template <int DIM, int NS, int STENCIL>
__global__ void __launch_bounds__(1024)
k_overlap(StepParams p, const InstInfo *__restrict__ inst, const float4 *__restrict__ Ps,
          const uint32_t *__restrict__ Is, const uint32_t *__restrict__ start,
          float4 *__restrict__ Pout, uint32_t *__restrict__ Iout, uint32_t *__restrict__ count,
          uint32_t *__restrict__ tile_cnt, uint32_t *__restrict__ flags) {
    __shared__ SpTab tab;
    load_tab(p, tab);
    __syncthreads();
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int i = blk * blockDim.x + threadIdx.x;
    if (i >= p.n_total) return;
    const float4 pi = Ps[i];
    const int si = species_of(pi.w);
    const InstInfo ii = inst[inst_of(pi.w)];
    OverlapVisitor ov{tab.share + si * p.n_species, {0.f, 0.f, 0.f}};
    pair_loop<DIM, NS, STENCIL>(p, tab, Ps, start, ii.bin_base, pi, si, ov);
    uint32_t flag = 0;
    float4 xn;
    xn.x = boundary(p, pi.x + ov.C[0], flag);
    xn.y = boundary(p, pi.y + ov.C[1], flag);
    xn.z = DIM == 3 ? boundary(p, pi.z + ov.C[2], flag) : 0.0f;
    xn.w = pi.w;
    if (!(isfinite(xn.x) && isfinite(xn.y) && isfinite(xn.z))) flag |= FLAG_NONFINITE;
    Pout[i] = xn;
    Iout[i] = Is[i];
    const uint32_t b = ii.bin_base + agent_bin<DIM>(p, xn);
    count_bin(count, tile_cnt, b, p.tile_totals, p.tile_reps);
    if (flag) atomicOr(flags, flag);
}

__global__ void k_set_u32(uint32_t *ptr, uint32_t v) { *ptr = v; }

__global__ void k_copy_f32(float *__restrict__ d, const float *__restrict__ s, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = s[i];
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
static inline unsigned grid_for(int64_t n, int block) {
    return (unsigned)((n + block - 1) / block);
}

void launch_init_agents(const StepParams &p, const Buffers &b, const float *x, const uint8_t *sp,
                        int write_species, hipStream_t s) {
    hipLaunchKernelGGL(k_init_agents, dim3(grid_for(p.n_total, 256)), dim3(256), 0, s, p,
                       b.inst, x, sp, b.species_id, write_species, b.P[0], b.I[0], b.flags);
}

void launch_bin(const StepParams &p, const Buffers &b, int src, int block, hipStream_t s) {
    const dim3 g(grid_for(p.n_total, block)), t(block);
    if (p.dim == 2)
        hipLaunchKernelGGL(k_bin<2>, g, t, 0, s, p, b.inst, b.P[src], b.count,
                           b.tile_cnt);
    else
        hipLaunchKernelGGL(k_bin<3>, g, t, 0, s, p, b.inst, b.P[src], b.count,
                           b.tile_cnt);
}

void launch_scan(const StepParams &p, const Buffers &b, int64_t n_bins_total, hipStream_t s) {
    const int64_t n = n_bins_total + 1;  // count[n_bins_total] is always 0
    const int T = (int)((n + kScanTile - 1) / kScanTile);
    if (!p.tile_totals)
        hipLaunchKernelGGL(k_tile_sums, dim3(T), dim3(256), 0, s, b.count, n, b.tile_cnt);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, b.tile_cnt, b.tile_sum, T,
                       p.tile_totals ? p.tile_reps : 1);
    hipLaunchKernelGGL(k_scan_apply, dim3(T), dim3(256), 0, s, b.count, n, b.tile_sum, b.start, T,
                       (uint32_t)p.n_total);
}

void launch_scatter(const StepParams &p, const Buffers &b, int src, int dst, int block,
                    hipStream_t s) {
    const dim3 g(grid_for(p.n_total, block)), t(block);
    if (p.dim == 2)
        hipLaunchKernelGGL(k_scatter<2>, g, t, 0, s, p, b.P[src], b.I[src], b.count, b.start,
                           b.P[dst], b.I[dst]);
    else
        hipLaunchKernelGGL(k_scatter<3>, g, t, 0, s, p, b.P[src], b.I[src], b.count, b.start,
                           b.P[dst], b.I[dst]);
}

void launch_stable(const StepParams &p, const Buffers &b, int src, int dst, int block,
                   hipStream_t s) {
    const dim3 g(grid_for(p.n_total, block)), t(block);
    if (p.dim == 2)
        hipLaunchKernelGGL(k_stable<2>, g, t, 0, s, p, b.inst, b.P[src], b.I[src], b.start,
                           b.P[dst], b.I[dst]);
    else
        hipLaunchKernelGGL(k_stable<3>, g, t, 0, s, p, b.inst, b.P[src], b.I[src], b.start,
                           b.P[dst], b.I[dst]);
}

// dynamic LDS of k_update: the pair walk's row table, a word per stencil
// row (9 in 3D, 3 in 2D) and thread
template <int DIM, int ST>
static size_t upd_lds(int block) {
    return ST == 3 ? (size_t)(DIM == 3 ? 36 : 12) * (size_t)block : 0;
}

template <int DIM, int NS, int ST>
static void upd(const StepParams &p, const Buffers &b, int src, int dst, int cbuf, int block,
                hipStream_t s) {
    hipLaunchKernelGGL((k_update<DIM, NS, ST, 0>), dim3(grid_for(p.n_total, block)), dim3(block),
                       (upd_lds<DIM, ST>(block)), s, p, b.inst, b.P[src], b.I[src], b.start, b.c[cbuf], b.P[dst],
                       b.I[dst], b.count, b.tile_cnt, b.step, b.flags);
}

// the exponential potential with the species specialisations of the
// harmonic one
template <int DIM, int NS, int ST>
static void upd_exp(const StepParams &p, const Buffers &b, int src, int dst, int cbuf, int block,
                    hipStream_t s) {
    hipLaunchKernelGGL((k_update<DIM, NS, ST, 1>), dim3(grid_for(p.n_total, block)), dim3(block),
                       (upd_lds<DIM, ST>(block)), s, p, b.inst, b.P[src], b.I[src], b.start, b.c[cbuf], b.P[dst],
                       b.I[dst], b.count, b.tile_cnt, b.step, b.flags);
}

// the hard-sphere overlap pass with the species specialisations of the pair
// loop (its share table stays in LDS: it is read only for overlapping pairs)
template <int DIM, int NS, int ST>
static void ovl(const StepParams &p, const Buffers &b, int src, int dst, int block,
                hipStream_t s) {
    hipLaunchKernelGGL((k_overlap<DIM, NS, ST>), dim3(grid_for(p.n_total, block)), dim3(block),
                       0, s, p, b.inst, b.P[src], b.I[src], b.start, b.P[dst], b.I[dst],
                       b.count, b.tile_cnt, b.flags);
}

// hard spheres (and a harmonic k = 0) use the generic (LDS) species table
template <int DIM, int ST, int POT>
static void upd_pot(const StepParams &p, const Buffers &b, int src, int dst, int cbuf, int block,
                    hipStream_t s) {
    hipLaunchKernelGGL((k_update<DIM, 0, ST, POT>), dim3(grid_for(p.n_total, block)),
                       dim3(block), (upd_lds<DIM, ST>(block)), s, p, b.inst, b.P[src], b.I[src], b.start, b.c[cbuf],
                       b.P[dst], b.I[dst], b.count, b.tile_cnt, b.step,
                       b.flags);
}

template <int DIM, int NS, int ST>
static void dbg(const StepParams &p, const Buffers &b, int src, uint32_t *count,
                unsigned long long *hash, float *F, int block, hipStream_t s) {
    if (p.potential == 0)
        hipLaunchKernelGGL((k_debug_pairs<DIM, NS, ST, 0>), dim3(grid_for(p.n_total, block)),
                           dim3(block), (upd_lds<DIM, ST>(block)), s, p, b.inst, b.P[src], b.I[src], b.start, count, hash,
                           F);
    else if (p.potential == 1)
        hipLaunchKernelGGL((k_debug_pairs<DIM, 0, ST, 1>), dim3(grid_for(p.n_total, block)),
                           dim3(block), (upd_lds<DIM, ST>(block)), s, p, b.inst, b.P[src], b.I[src], b.start, count, hash,
                           F);
    else
        hipLaunchKernelGGL((k_debug_pairs<DIM, 0, ST, 2>), dim3(grid_for(p.n_total, block)),
                           dim3(block), (upd_lds<DIM, ST>(block)), s, p, b.inst, b.P[src], b.I[src], b.start, count, hash,
                           F);
}

#define PC_DISPATCH(FN, ...)                                                        \
    do {                                                                            \
        const int ns = p.n_species == 1 ? 1 : (p.n_species == 2 ? 2 : 0);           \
        if (p.dim == 2) {                                                           \
            if (p.stencil == 3) {                                                   \
                if (ns == 1) FN<2, 1, 3>(__VA_ARGS__);                              \
                else if (ns == 2) FN<2, 2, 3>(__VA_ARGS__);                         \
                else FN<2, 0, 3>(__VA_ARGS__);                                      \
            } else {                                                                \
                if (ns == 1) FN<2, 1, 2>(__VA_ARGS__);                              \
                else if (ns == 2) FN<2, 2, 2>(__VA_ARGS__);                         \
                else FN<2, 0, 2>(__VA_ARGS__);                                      \
            }                                                                       \
        } else {                                                                    \
            if (p.stencil == 3) {                                                   \
                if (ns == 1) FN<3, 1, 3>(__VA_ARGS__);                              \
                else if (ns == 2) FN<3, 2, 3>(__VA_ARGS__);                         \
                else FN<3, 0, 3>(__VA_ARGS__);                                      \
            } else {                                                                \
                if (ns == 1) FN<3, 1, 2>(__VA_ARGS__);                              \
                else if (ns == 2) FN<3, 2, 2>(__VA_ARGS__);                         \
                else FN<3, 0, 2>(__VA_ARGS__);                                      \
            }                                                                       \
        }                                                                           \
    } while (0)

void launch_update(const StepParams &p, const Buffers &b, int src, int dst, int cbuf, int block,
                   hipStream_t s) {
    // the harmonic pair loop needs k > 0 (its force factor is 0 * inf at
    // r = 0 when k = 0); with k = 0 the pair-free variant gives the same bits
    if (p.potential == 0 && p.k != 0.0f) {
        PC_DISPATCH(upd, p, b, src, dst, cbuf, block, s);
        return;
    }
    if (p.potential == 1) {
        PC_DISPATCH(upd_exp, p, b, src, dst, cbuf, block, s);
        return;
    }
#define PC_POT(D, S) upd_pot<D, S, 2>(p, b, src, dst, cbuf, block, s)
    if (p.dim == 2) {
        if (p.stencil == 3) PC_POT(2, 3);
        else PC_POT(2, 2);
    } else {
        if (p.stencil == 3) PC_POT(3, 3);
        else PC_POT(3, 2);
    }
#undef PC_POT
}

void launch_overlap(const StepParams &p, const Buffers &b, int src, int dst, int block,
                    hipStream_t s) {
    PC_DISPATCH(ovl, p, b, src, dst, block, s);
}

void launch_debug_pairs(const StepParams &p, const Buffers &b, int src, uint32_t *count,
                        unsigned long long *hash, float *F, int block, hipStream_t s) {
    PC_DISPATCH(dbg, p, b, src, count, hash, F, block, s);
}

template <int DIM, int NS, bool UPT>
static void dep(const StepParams &p, const Buffers &b, int src, hipStream_t s) {
    if (p.deposit_agg)
        hipLaunchKernelGGL((k_deposit<DIM, NS, UPT, true>), dim3(grid_for(p.n_total, 1024)),
                           dim3(1024), 0, s, p, b.inst, b.P[src], b.S_src, b.S_upt);
    else
        hipLaunchKernelGGL((k_deposit<DIM, NS, UPT, false>), dim3(grid_for(p.n_total, 256)),
                           dim3(256), 0, s, p, b.inst, b.P[src], b.S_src, b.S_upt);
}

void launch_deposit(const StepParams &p, const Buffers &b, int src, hipStream_t s) {
    const int ns = p.n_species == 1 ? 1 : (p.n_species == 2 ? 2 : 0);
#define PC_DEP(D, N)                                  \
    do {                                              \
        if (p.has_uptake) dep<D, N, true>(p, b, src, s);  \
        else dep<D, N, false>(p, b, src, s);          \
    } while (0)
    if (p.dim == 2) {
        if (ns == 1) PC_DEP(2, 1);
        else if (ns == 2) PC_DEP(2, 2);
        else PC_DEP(2, 0);
    } else {
        if (ns == 1) PC_DEP(3, 1);
        else if (ns == 2) PC_DEP(3, 2);
        else PC_DEP(3, 0);
    }
#undef PC_DEP
}

template <int DIM, int NS, bool UPT>
static void chem(const StepParams &p, const PdeParams &q, const Buffers &b, int src, int cur,
                 int n_sub, hipStream_t s) {
    const size_t lds = 8 * (size_t)q.nodes_per_inst * (UPT ? 2 : 1);
    // small grids (the 52^2 grids of the Fig. 1 ensemble) run faster with
    // 512 threads, larger ones (128^2) with 1024
    const int threads = q.nodes_per_inst <= 4096 ? 512 : 1024;
    hipLaunchKernelGGL((k_chem_inst<DIM, NS, UPT>), dim3(p.n_inst), dim3(threads), lds, s, p, q,
                       b.inst, b.P[src], b.c[0], b.c[1], cur, n_sub, b.flags, b.step);
}

size_t chem_inst_lds_bytes(const PdeParams &q) {
    return 8 * (size_t)q.nodes_per_inst * (q.has_uptake ? 2 : 1);
}

void launch_chem_inst(const StepParams &p, const PdeParams &q, const Buffers &b, int src, int cur,
                      int n_sub, hipStream_t s) {
    const int ns = p.n_species == 1 ? 1 : (p.n_species == 2 ? 2 : 0);
#define PC_CHEM(D, N)                                                   \
    do {                                                                \
        if (p.has_uptake) chem<D, N, true>(p, q, b, src, cur, n_sub, s); \
        else chem<D, N, false>(p, q, b, src, cur, n_sub, s);            \
    } while (0)
    if (p.dim == 2) {
        if (ns == 1) PC_CHEM(2, 1);
        else if (ns == 2) PC_CHEM(2, 2);
        else PC_CHEM(2, 0);
    } else {
        if (ns == 1) PC_CHEM(3, 1);
        else if (ns == 2) PC_CHEM(3, 2);
        else PC_CHEM(3, 0);
    }
#undef PC_CHEM
}

// k_pde launch shape: one work-group per x-row of the grid, its width
// rounded up to whole waves (at most 256 threads; longer rows loop)
static dim3 pde_grid(const PdeParams &q) { return dim3((uint32_t)(q.n_nodes_total / q.grid_n)); }
static dim3 pde_block(const PdeParams &q) { return dim3(std::min(256, (q.grid_n + 63) / 64 * 64)); }

void launch_pde(const PdeParams &q, const Buffers &b, int cin, int cout, int last,
                hipStream_t s) {
    const dim3 g = pde_grid(q), t = pde_block(q);
    if (q.kde) {
        if (q.dim == 2)
            hipLaunchKernelGGL((k_pde<2, true>), g, t, 0, s, q, b.c[cin], b.c[cout], b.S_src,
                               b.S_upt, last, b.flags,
                               last ? b.step : nullptr);
        else
            hipLaunchKernelGGL((k_pde<3, true>), g, t, 0, s, q, b.c[cin], b.c[cout], b.S_src,
                               b.S_upt, last, b.flags,
                               last ? b.step : nullptr);
        return;
    }
    if (q.dim == 2)
        hipLaunchKernelGGL((k_pde<2, false>), g, t, 0, s, q, b.c[cin], b.c[cout], b.S_src,
                           b.S_upt, last, b.flags, last ? b.step : nullptr);
    else
        hipLaunchKernelGGL((k_pde<3, false>), g, t, 0, s, q, b.c[cin], b.c[cout], b.S_src,
                           b.S_upt, last, b.flags, last ? b.step : nullptr);
}

void launch_pde_ptr(const PdeParams &q, const float *cin, float *cout, unsigned long long *Ssrc,
                    unsigned long long *Supt, int last, uint32_t *flags, hipStream_t s) {
    const dim3 g = pde_grid(q), t = pde_block(q);
    if (q.dim == 2)
        hipLaunchKernelGGL((k_pde<2, false>), g, t, 0, s, q, cin, cout, Ssrc, Supt, last, flags,
                           nullptr);
    else
        hipLaunchKernelGGL((k_pde<3, false>), g, t, 0, s, q, cin, cout, Ssrc, Supt, last, flags,
                           nullptr);
}


void launch_zero_u32(uint32_t *d, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_zero_u32, dim3(grid_for(n, 256)), dim3(256), 0, s, d, n);
}

void launch_positions(const StepParams &p, const Buffers &b, int src, float *out,
                      hipStream_t s) {
    hipLaunchKernelGGL(k_positions, dim3(grid_for(p.n_total, 256)), dim3(256), 0, s, p, b.inst,
                       b.P[src], b.I[src], out);
}

void launch_species(const StepParams &p, const Buffers &b, int src, uint8_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_species, dim3(grid_for(p.n_total, 256)), dim3(256), 0, s, p, b.inst,
                       b.P[src], b.I[src], out);
}

void launch_apply_species(const StepParams &p, const Buffers &b, int src, const uint8_t *sp,
                          hipStream_t s) {
    hipLaunchKernelGGL(k_apply_species, dim3(grid_for(p.n_total, 256)), dim3(256), 0, s, p,
                       b.inst, b.P[src], b.I[src], sp, b.flags);
}

void launch_set_u32(uint32_t *ptr, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, ptr, v);
}

void launch_copy_f32(float *dst, const float *src, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy_f32, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, src, n);
}

}  // namespace pc
