// Owner-computes particle-in-cell deposit (and, with one PDE substep, the
// PDE update) for gfx950: one work-group per slab of grid nodes, no device
// atomics.
//
// The deposit of eq. random_measure spreads each agent's source and uptake
// over the 2^dim corners of its grid cell with piecewise-linear weights
// (Sect. 2.3).  Scattered from the agents, each corner is a device atomic,
// and MI355X serves device atomics one 64-byte line at a time beyond the
// L2s, so a million agents' scattered adds cost tens of microseconds.  Here
// a work-group owns a slab of nodes: whole rows along x, By rows along y
// (and Bz layers along z).  With the step's new positions sorted by bin
// (the step sorts X^{n+1} before the deposit), the agents whose cells touch
// the slab lie in the bin rows of a range of y for each z of a range: in
// the row-major bin order each such z layer is one contiguous run of the
// sorted agents.  The work-group lays its few runs end to end, every thread
// takes eight consecutive agents from them, sums the corners that fall in
// its slab per cell in registers and adds them to LDS sums, and then stores
// each owned node's sums once or, when the step has a single PDE substep,
// applies the forward-Euler update of eq. pde_c to its owned nodes
// directly (the sums never reach HBM).  Each corner is added by exactly one
// work-group, so every node receives the same integer as on every other
// deposit path (fixed point, 2^-32 units, charge times the axis weights in
// axis order), and the PDE node update is the same function as k_pde's.
//
// One work-group per slab serialises where chemotaxis has collapsed a blob
// into a few cells: a slab can then hold 10^5 agents.  A slab with more
// agents than a threshold is handed over: its run table is recorded and its
// nodes' deposits zeroed, its agents are spread in chunks over many
// work-groups (each sums a chunk's owned corners in LDS and adds the nonzero
// node sums to HBM with device atomics), and k_slab_finish applies the PDE
// to its nodes.  The sums are still integers, so the bits do not depend on
// which slabs were handed over.  In the step the hand-over runs in the
// scatter's grid (k_scatter_classify: it needs only the bin starts), and the
// light slabs' work-groups and the assisting ones share one grid
// (k_slab_merged), so that their work overlaps; no work-group ever waits on
// another inside a kernel.  k_chem_slabs and k_slab_assist are the same
// bodies launched one after the other.
#include "pc_device.h"

namespace pc {

constexpr int kSlabRuns = 256;   // contiguous agent runs per slab (LDS table)
constexpr int kSlabThreads = kSlabRuns;   // one run lookup per thread
// per-slab run table handed to k_slab_assist: run count, run starts, prefixes
constexpr int kSlabTableWords = 2 * kSlabRuns + 2;
constexpr int kAssistChunk = 1024;   // agents of a heavy slab per assisting pass
constexpr int kAssistThreads = 256;
static_assert(kAssistThreads == kSlabThreads, "k_slab_merged runs both kinds of work-group");
constexpr int kAssistBlocks = 1024;   // grid when the occupancy query fails
constexpr int kAssistSlabBlock = 4 * kAssistThreads;   // slab counts scanned per pass
constexpr int kFinishParts = 4;   // work-groups per handed-over slab in k_slab_finish

// Bins holding every agent whose cell lies in [c0, c1] along one axis, as
// up to two disjoint inclusive intervals (c0 = -1 on the torus: cell n - 1
// through the seam).  An agent of cell c sits in [c h, (c + 1) h] up to a
// few float32 ulps, so its bin floor(x nb / L) lies within 1e-3 of a bin of
// the exact range; the margin covers that and nothing more.
struct Span {
    int lo[2], hi[2];
    int k;
};

__device__ __forceinline__ void bins_of_cells(const StepParams &p, int c0, int c1, Span &s) {
    const int nb = p.nb;
    const float f = p.h * p.inv_bin;   // bins per cell
    auto iv = [&](int a, int b, int &lo, int &hi) {
        lo = max((int)floorf((float)a * f - 1e-3f), 0);
        hi = min((int)floorf((float)(b + 1) * f + 1e-3f), nb - 1);
    };
    s.k = 1;
    iv(max(c0, 0), c1, s.lo[0], s.hi[0]);
    if (c0 < 0) {
        int wl, wh;
        iv(p.grid_n - 1, p.grid_n - 1, wl, wh);
        if (wl <= s.hi[0] + 1) {
            s.hi[0] = max(s.hi[0], wh);
        } else {
            s.lo[1] = wl;
            s.hi[1] = wh;
            s.k = 2;
        }
    }
}

// Cells feeding the owned nodes [o0, o1) along one axis: node i takes cells
// i - 1 and i (torus: mod n; walls: cells 0 .. n - 2 only).
__device__ __forceinline__ void cells_of_nodes(const StepParams &p, int o0, int o1, int &c0,
                                               int &c1) {
    c0 = o0 - 1;
    c1 = o1 - 1;
    if (!p.periodic) {
        c0 = max(c0, 0);
        c1 = min(c1, p.grid_n - 2);
    }
}

// Owned nodes of slab s: instance k, y rows [y0, y1), z layers [z0, z1),
// all x.
struct SlabGeom {
    int k, y0, y1, z0, z1, owned;
};

template <int DIM>
__device__ __forceinline__ SlabGeom slab_geom(int s, int n, int By, int Bz, int nby, int nbz) {
    SlabGeom g;
    const int per_inst = nby * nbz;
    g.k = s / per_inst;
    const int bl = s - g.k * per_inst;
    const int jy = bl % nby, jz = bl / nby;
    g.y0 = jy * By;
    g.y1 = min(g.y0 + By, n);
    g.z0 = DIM == 3 ? jz * Bz : 0;
    g.z1 = DIM == 3 ? min(g.z0 + Bz, n) : 1;
    g.owned = n * (g.y1 - g.y0) * (g.z1 - g.z0);
    return g;
}

// Corner sums of a run of agents in one cell, kept in registers and added
// to the LDS sums when the cell changes: agents in cell order repeat their
// cell, and inside a collapsed blob every lane of a wave would otherwise
// add to the same few LDS words.  Each corner value is the fixed-point
// integer of the charge times the axis weights in axis order, as on every
// deposit path, so sums of them are the same integers in any grouping.
template <int DIM, int NS, bool UPT>
struct SlabAcc {
    int key;                      // cell of the held sums (-1: none)
    int l[1 << DIM];              // their owned-node indices (-1: not owned)
    unsigned long long s[1 << DIM], u[1 << DIM];

    __device__ __forceinline__ void init() { key = -1; }

    __device__ __forceinline__ void flush(unsigned long long *sums, int owned) {
        if (key < 0) return;
#pragma unroll
        for (int m = 0; m < (1 << DIM); ++m) {
            if (l[m] < 0) continue;
            if (s[m]) atomicAdd(&sums[l[m]], s[m]);
            if (UPT && u[m]) atomicAdd(&sums[owned + l[m]], u[m]);
        }
        key = -1;
    }

    __device__ __forceinline__ void add(const StepParams &p, const SpTab &tab, const float4 x,
                                        const SlabGeom &g, unsigned long long *sums) {
        const int n = p.grid_n;
        const int sp = species_of(x.w);
        const float qs = sel<NS>(p.src_fx, tab.src, sp);
        const float qu = UPT ? sel<NS>(p.upt_fx, tab.upt, sp) : 0.0f;
        if (qs == 0.0f && qu == 0.0f) return;
        Cell cc[3];
        cc[0] = cell_of(p, x.x);
        cc[1] = cell_of(p, x.y);
        cc[2] = Cell{0, 0, 0.0f};
        if (DIM == 3) cc[2] = cell_of(p, x.z);
        const int k = cc[0].i0 + n * (cc[1].i0 + n * cc[2].i0);
        if (k != key) {
            flush(sums, g.owned);
            key = k;
            const int ly0 = cc[1].i0 - g.y0, ly1 = cc[1].i1 - g.y0;
            const int oy[2] = {(ly0 >= 0 && ly0 < g.y1 - g.y0) ? ly0 : -1,
                               (ly1 >= 0 && ly1 < g.y1 - g.y0) ? ly1 : -1};
            int oz[2] = {0, -1};
            if (DIM == 3) {
                const int lz0 = cc[2].i0 - g.z0, lz1 = cc[2].i1 - g.z0;
                oz[0] = (lz0 >= 0 && lz0 < g.z1 - g.z0) ? lz0 : -1;
                oz[1] = (lz1 >= 0 && lz1 < g.z1 - g.z0) ? lz1 : -1;
            }
            const int ny = g.y1 - g.y0;
#pragma unroll
            for (int m = 0; m < (1 << DIM); ++m) {
                const int ux = m & 1, uy = (m >> 1) & 1, uz = (m >> 2) & 1;
                l[m] = (oy[uy] < 0 || oz[uz] < 0) ? -1
                                                  : (ux ? cc[0].i1 : cc[0].i0) + n * (oy[uy] + ny * oz[uz]);
                s[m] = 0ull;
                u[m] = 0ull;
            }
        }
#pragma unroll
        for (int m = 0; m < (1 << DIM); ++m) {
            const int ux = m & 1, uy = (m >> 1) & 1, uz = (m >> 2) & 1;
            // the charge times the axis weights in axis order, as every
            // deposit path forms it
            float ws = qs, wu = qu;
            const float fx = ux ? cc[0].t : 1.0f - cc[0].t;
            const float fy = uy ? cc[1].t : 1.0f - cc[1].t;
            ws *= fx;
            if (UPT) wu *= fx;
            ws *= fy;
            if (UPT) wu *= fy;
            if (DIM == 3) {
                const float fz = uz ? cc[2].t : 1.0f - cc[2].t;
                ws *= fz;
                if (UPT) wu *= fz;
            }
            s[m] += (unsigned long long)__float2ull_rn(ws);
            if (UPT) u[m] += (unsigned long long)__float2ull_rn(wu);
        }
    }
};

// Agents [a, e) of a slab's runs laid end to end (run_a: run starts in the
// cell list, run_pre: exclusive prefixes of the run lengths), kPer
// consecutive agents per thread and pass: their loads are issued together,
// then they are summed per cell in registers and added to the LDS sums.
template <int DIM, int NS, bool UPT, int kPer>
__device__ __forceinline__ void slab_run_agents(const StepParams &p, const SpTab &tab,
                                                const float4 *__restrict__ Ps,
                                                const uint32_t *run_a, const uint32_t *run_pre,
                                                int nrun, uint32_t a, uint32_t e,
                                                const SlabGeom &g, unsigned long long *sums) {
    SlabAcc<DIM, NS, UPT> acc;
    acc.init();
    for (uint32_t w0 = a + threadIdx.x * (uint32_t)kPer; w0 < e;
         w0 += blockDim.x * (uint32_t)kPer) {
        int r0 = 0, r1 = nrun - 1;   // the run holding w0
        while (r0 < r1) {
            const int mid = (r0 + r1 + 1) >> 1;
            if (run_pre[mid] <= w0) r0 = mid;
            else r1 = mid - 1;
        }
        float4 xs[kPer];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            const uint32_t w = w0 + (uint32_t)k;
            xs[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (w < e) {
                while (r0 + 1 < nrun && run_pre[r0 + 1] <= w) ++r0;
                xs[k] = Ps[run_a[r0] + (w - run_pre[r0])];
            }
        }
#pragma unroll
        for (int k = 0; k < kPer; ++k)
            if (w0 + (uint32_t)k < e) acc.add(p, tab, xs[k], g, sums);
    }
    acc.flush(sums, g.owned);
}

template <int DIM>
__device__ __forceinline__ int64_t slab_node(const SlabGeom &g, const InstInfo &ii, int n, int l,
                                             int ic[3]) {
    const int ny = g.y1 - g.y0;
    ic[0] = l % n;
    ic[1] = g.y0 + (l / n) % ny;
    ic[2] = g.z0 + l / (n * ny);
    return (int64_t)ii.node_base + ic[0] + (int64_t)n * (ic[1] + (int64_t)n * ic[2]);
}

// The PDE substep at the slab's owned nodes from their deposits (with
// BY_NODE, HBM arrays indexed by node; else the LDS sums indexed by owned
// node), two nodes per thread and pass: the second node's index is clamped
// so that both stencils load unconditionally and only its store is guarded.
template <int DIM, bool UPT, bool BY_NODE>
__device__ __forceinline__ void slab_pde_nodes(const PdeParams &q, const SlabGeom &g,
                                               const InstInfo &ii, int n,
                                               const float *__restrict__ cin,
                                               float *__restrict__ cout,
                                               const unsigned long long *sS,
                                               const unsigned long long *sU, int lbeg, int lend,
                                               uint32_t &flag) {
    for (int l0 = lbeg + threadIdx.x; l0 < lend; l0 += 2 * blockDim.x) {
        const int l1 = l0 + (int)blockDim.x;
        const bool two = l1 < lend;
        const int l1c = two ? l1 : l0;
        int ic0[3], ic1[3];
        const int64_t n0 = slab_node<DIM>(g, ii, n, l0, ic0);
        const int64_t n1 = slab_node<DIM>(g, ii, n, l1c, ic1);
        const int64_t k0 = BY_NODE ? n0 : l0, k1 = BY_NODE ? n1 : l1c;
        const unsigned long long s0 = sS[k0], s1 = sS[k1];
        const unsigned long long u0 = UPT ? sU[k0] : 0ull, u1 = UPT ? sU[k1] : 0ull;
        const float v0 = pde_node<DIM>(q, cin + ii.node_base, ic0, s0, u0, flag);
        const float v1 = pde_node<DIM>(q, cin + ii.node_base, ic1, s1, u1, flag);
        cout[n0] = v0;
        if (two) cout[n1] = v1;
    }
}

// One work-group's slab.  PART 0: everything (a heavy slab handed over,
// a light one deposited and updated); PART 1: only the classification and
// the hand-over of heavy slabs (slab_cnt, run table, zeroed deposits);
// PART 2: only the light slabs (the heavy ones were handed over by PART 1).
template <int DIM, int NS, bool UPT, int PART>
__device__ __forceinline__ void chem_slab_body(
    const StepParams &p, const PdeParams &q, const InstInfo *__restrict__ inst,
    const float4 *__restrict__ Ps, const uint32_t *__restrict__ start,
    const float *__restrict__ cin, float *__restrict__ cout,
    unsigned long long *__restrict__ Ssrc, unsigned long long *__restrict__ Supt, int By,
    int Bz, int nby, int nbz, int fuse_pde, uint32_t split, uint32_t *__restrict__ slab_cnt,
    uint32_t *__restrict__ slab_tab, uint32_t *__restrict__ flags, int slab) {
    extern __shared__ unsigned long long sums[];   // owned source sums, then uptake
    __shared__ uint32_t run_a[kSlabRuns];
    __shared__ uint32_t run_pre[kSlabRuns + 1];
    __shared__ uint32_t wtot[kSlabRuns / 64];
    __shared__ SpTab tab;
    const int n = p.grid_n;
    const int nb = p.nb;
    const SlabGeom g = slab_geom<DIM>(slab, n, By, Bz, nby, nbz);
    const int y0 = g.y0, y1 = g.y1, z0 = g.z0, z1 = g.z1, owned = g.owned;
    const InstInfo ii = inst[g.k];
    if (PART != 1)
        for (int l = threadIdx.x; l < owned * (UPT ? 2 : 1); l += blockDim.x) sums[l] = 0ull;
    if (NS == 0 && PART != 1) load_tab(p, tab);
    // runs: one per z bin layer of the box and y interval, holding all x bins
    // of that y interval (contiguous in the row-major bin order); one thread
    // per run looks up its bounds, then the lengths are scanned
    Span sy, sz;
    {
        int c0, c1;
        cells_of_nodes(p, y0, y1, c0, c1);
        bins_of_cells(p, c0, c1, sy);
        if (DIM == 3) {
            cells_of_nodes(p, z0, z1, c0, c1);
            bins_of_cells(p, c0, c1, sz);
        } else {
            sz.k = 1;
            sz.lo[0] = sz.hi[0] = 0;
        }
    }
    const int nz0 = sz.hi[0] - sz.lo[0] + 1;
    const int nzl = nz0 + (sz.k == 2 ? sz.hi[1] - sz.lo[1] + 1 : 0);
    int nrun = nzl * sy.k;
    if (nrun > kSlabRuns) {
        // the host sizes slabs so this cannot happen; report it rather than
        // drop agents silently
        if (threadIdx.x == 0) atomicOr(flags, FLAG_INTERNAL);
        nrun = kSlabRuns;
    }
    uint32_t len = 0;
    if ((int)threadIdx.x < nrun) {
        const int iy = threadIdx.x % sy.k, li = threadIdx.x / sy.k;
        const int bz = li < nz0 ? sz.lo[0] + li : sz.lo[1] + (li - nz0);
        const int ylo = iy ? sy.lo[1] : sy.lo[0], yhi = iy ? sy.hi[1] : sy.hi[0];
        const uint32_t row0 = ii.bin_base + (uint32_t)((bz * nb + ylo) * nb);
        const uint32_t row1 = ii.bin_base + (uint32_t)((bz * nb + yhi + 1) * nb);
        const uint32_t a = start[row0];
        run_a[threadIdx.x] = a;
        len = start[row1] - a;
    }
    // exclusive scan of the run lengths over the first kSlabRuns threads
    // (four waves)
    if (threadIdx.x < kSlabRuns) {
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        uint32_t x = len;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (lane == 63) wtot[wv] = x;
        run_pre[threadIdx.x] = x - len;   // wave-local for now
    }
    __syncthreads();
    if (threadIdx.x < kSlabRuns) {
        uint32_t base = 0;
        for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) base += wtot[w];
        run_pre[threadIdx.x] += base;
        if ((int)threadIdx.x == kSlabRuns - 1)
            run_pre[kSlabRuns] = base + wtot[kSlabRuns / 64 - 1];
    }
    __syncthreads();
    const uint32_t total = run_pre[nrun];
    const bool heavy = total > split;
    if (PART != 2 && threadIdx.x == 0) slab_cnt[slab] = heavy ? total : 0u;
    if (heavy) {
        if (PART == 2) return;   // handed over before this kernel
        // handed over: the run table for the assisting work-groups, and
        // zeroed deposits for their atomics
        uint32_t *T = slab_tab + (size_t)slab * kSlabTableWords;
        if (threadIdx.x == 0) T[0] = (uint32_t)nrun;
        for (int t = threadIdx.x; t <= nrun; t += blockDim.x) {
            if (t < nrun) T[1 + t] = run_a[t];
            T[1 + kSlabRuns + t] = run_pre[t];
        }
        int ic[3];
        for (int l = threadIdx.x; l < owned; l += blockDim.x) {
            const int64_t node = slab_node<DIM>(g, ii, n, l, ic);
            Ssrc[node] = 0ull;
            if (UPT) Supt[node] = 0ull;
        }
        return;
    }
    if (PART == 1) return;   // a light slab: the next kernel's
    slab_run_agents<DIM, NS, UPT, 8>(p, tab, Ps, run_a, run_pre, nrun, 0u, total, g, sums);
    __syncthreads();
    uint32_t flag = 0;
    if (fuse_pde) {
        slab_pde_nodes<DIM, UPT, false>(q, g, ii, n, cin, cout, sums, sums + owned, 0, owned,
                                        flag);
    } else {
        int ic[3];
        for (int l = threadIdx.x; l < owned; l += blockDim.x) {
            const int64_t node = slab_node<DIM>(g, ii, n, l, ic);
            Ssrc[node] = sums[l];
            if (UPT) Supt[node] = sums[owned + l];
        }
    }
    if (flag) atomicOr(flags, flag);
}

template <int DIM, int NS, bool UPT>
__global__ void __launch_bounds__(kSlabThreads)
k_chem_slabs(StepParams p, PdeParams q, const InstInfo *__restrict__ inst,
             const float4 *__restrict__ Ps, const uint32_t *__restrict__ start,
             const float *__restrict__ cin, float *__restrict__ cout,
             unsigned long long *__restrict__ Ssrc, unsigned long long *__restrict__ Supt,
             int By, int Bz, int nby, int nbz, int fuse_pde, uint32_t split,
             uint32_t *__restrict__ slab_cnt, uint32_t *__restrict__ slab_tab,
             uint32_t *__restrict__ flags, uint32_t *__restrict__ stepc) {
    // with the PDE fused, this kernel advances the step counter: the update,
    // which reads it, has finished, and nothing after it in the step reads it
    if (fuse_pde && stepc && blockIdx.x == 0 && threadIdx.x == 0) *stepc += 1u;
    chem_slab_body<DIM, NS, UPT, 0>(p, q, inst, Ps, start, cin, cout, Ssrc, Supt, By, Bz, nby,
                                    nbz, fuse_pde, split, slab_cnt, slab_tab, flags,
                                    (int)blockIdx.x);
}

// The agents of the handed-over slabs.  Slab s contributes ceil(cnt_s /
// kAssistChunk) chunks, numbered in slab order; assisting work-group b of G
// takes chunks b, b + G, ...  For a chunk it loads the slab's run table, sums the
// owned corners of the chunk's agents in LDS and adds each nonzero node sum
// to the slab's zeroed deposits with one device atomic.  Every work-group
// scans the slab counts itself (kAssistSlabBlock at a time), so no counter
// has to be reset between steps; with no handed-over slab it only reads the
// counts.
template <int DIM, int NS, bool UPT>
__device__ __forceinline__ void slab_assist_body(
    const StepParams &p, const InstInfo *__restrict__ inst, const float4 *__restrict__ Ps,
    unsigned long long *__restrict__ Ssrc, unsigned long long *__restrict__ Supt, int By,
    int Bz, int nby, int nbz, int nslabs, const uint32_t *__restrict__ slab_cnt,
    const uint32_t *__restrict__ slab_tab, uint32_t b, uint32_t G) {
    extern __shared__ unsigned long long sums[];
    __shared__ uint32_t pre[kAssistSlabBlock + 1];
    __shared__ uint32_t run_a[kSlabRuns];
    __shared__ uint32_t run_pre[kSlabRuns + 1];
    __shared__ uint32_t wtot[kAssistThreads / 64];
    __shared__ SpTab tab;
    if (NS == 0) load_tab(p, tab);
    const int n = p.grid_n;
    uint32_t base = 0;   // chunks of the slabs before this block of slabs
    for (int s0 = 0; s0 < nslabs; s0 += kAssistSlabBlock) {
        uint32_t c[4], loc = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int sl = s0 + (int)threadIdx.x * 4 + e;
            const uint32_t cnt = sl < nslabs ? slab_cnt[sl] : 0u;
            c[e] = (cnt + kAssistChunk - 1) / kAssistChunk;
            loc += c[e];
        }
        // block-wide exclusive scan of the per-thread chunk counts
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        uint32_t x = loc;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        if (lane == 63) wtot[wv] = x;
        __syncthreads();
        uint32_t wb = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < kAssistThreads / 64; ++w) {
            if (w < wv) wb += wtot[w];
            tot += wtot[w];
        }
        uint32_t run = base + wb + x - loc;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            pre[threadIdx.x * 4 + e] = run;
            run += c[e];
        }
        if (threadIdx.x == 0) pre[kAssistSlabBlock] = base + tot;
        __syncthreads();
        // this work-group's chunks among [base, base + tot)
        uint32_t ch = base + (b + G - base % G) % G;
        for (; ch < base + tot; ch += G) {
            // slab: the last j with pre[j] <= ch (pre is non-decreasing)
            int lo = 0, hi = kAssistSlabBlock - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (pre[mid] <= ch) lo = mid;
                else hi = mid - 1;
            }
            const int sl = s0 + lo;
            const uint32_t cnt = slab_cnt[sl];
            const uint32_t a0 = (ch - pre[lo]) * (uint32_t)kAssistChunk;
            const uint32_t a1 = min(a0 + (uint32_t)kAssistChunk, cnt);
            const SlabGeom g = slab_geom<DIM>(sl, n, By, Bz, nby, nbz);
            const InstInfo ii = inst[g.k];
            const uint32_t *T = slab_tab + (size_t)sl * kSlabTableWords;
            const int nrun = (int)T[0];
            for (int t = threadIdx.x; t < nrun; t += blockDim.x) run_a[t] = T[1 + t];
            for (int t = threadIdx.x; t <= nrun; t += blockDim.x) run_pre[t] = T[1 + kSlabRuns + t];
            for (int l = threadIdx.x; l < g.owned * (UPT ? 2 : 1); l += blockDim.x) sums[l] = 0ull;
            __syncthreads();
            slab_run_agents<DIM, NS, UPT, kAssistChunk / kAssistThreads>(p, tab, Ps, run_a,
                                                                        run_pre, nrun, a0, a1, g,
                                                                        sums);
            __syncthreads();
            int ic[3];
            for (int l = threadIdx.x; l < g.owned; l += blockDim.x) {
                const unsigned long long vS = sums[l], vU = UPT ? sums[g.owned + l] : 0ull;
                if (vS == 0ull && vU == 0ull) continue;
                const int64_t node = slab_node<DIM>(g, ii, n, l, ic);
                if (vS) atomicAdd(&Ssrc[node], vS);
                if (UPT && vU) atomicAdd(&Supt[node], vU);
            }
            __syncthreads();
        }
        base += tot;
        __syncthreads();   // pre and wtot are rewritten by the next block of slabs
    }
}

template <int DIM, int NS, bool UPT>
__global__ void __launch_bounds__(kAssistThreads)
k_slab_assist(StepParams p, const InstInfo *__restrict__ inst, const float4 *__restrict__ Ps,
              unsigned long long *__restrict__ Ssrc, unsigned long long *__restrict__ Supt,
              int By, int Bz, int nby, int nbz, int nslabs,
              const uint32_t *__restrict__ slab_cnt, const uint32_t *__restrict__ slab_tab) {
    slab_assist_body<DIM, NS, UPT>(p, inst, Ps, Ssrc, Supt, By, Bz, nby, nbz, nslabs, slab_cnt,
                                   slab_tab, blockIdx.x, gridDim.x);
}

// The hand-over alone: every slab classified (slab_cnt), the heavy ones'
// run tables written and deposits zeroed.
template <int DIM, int NS, bool UPT>
__global__ void __launch_bounds__(kSlabThreads)
k_slab_classify(StepParams p, PdeParams q, const InstInfo *__restrict__ inst,
                const float4 *__restrict__ Ps, const uint32_t *__restrict__ start,
                unsigned long long *__restrict__ Ssrc, unsigned long long *__restrict__ Supt,
                int By, int Bz, int nby, int nbz, uint32_t split,
                uint32_t *__restrict__ slab_cnt, uint32_t *__restrict__ slab_tab,
                uint32_t *__restrict__ flags) {
    chem_slab_body<DIM, NS, UPT, 1>(p, q, inst, Ps, start, nullptr, nullptr, Ssrc, Supt, By, Bz,
                                    nby, nbz, 0, split, slab_cnt, slab_tab, flags,
                                    (int)blockIdx.x);
}

// The counting sort's scatter of X^{n+1} and the slab classification in
// one grid: the first nsc work-groups scatter the agents, the rest classify
// the slabs (and hand the heavy ones over).  The classification reads only
// the bin starts, which the scan wrote before this kernel, and writes
// nothing the scatter reads.
template <int DIM, int NS, bool UPT>
__global__ void __launch_bounds__(kSlabThreads)
k_scatter_classify(StepParams p, PdeParams q, const InstInfo *__restrict__ inst,
                   const float4 *__restrict__ P, const uint32_t *__restrict__ I,
                   uint32_t *__restrict__ count, const uint32_t *__restrict__ start,
                   float4 *__restrict__ Ps, uint32_t *__restrict__ Is,
                   unsigned long long *__restrict__ Ssrc, unsigned long long *__restrict__ Supt,
                   int By, int Bz, int nby, int nbz, uint32_t split,
                   uint32_t *__restrict__ slab_cnt, uint32_t *__restrict__ slab_tab,
                   uint32_t *__restrict__ flags, uint32_t nsc) {
    if (blockIdx.x < nsc) {
        const uint32_t blk = xcd_block(blockIdx.x, nsc);
        const int i = blk * blockDim.x + threadIdx.x;
        if (i >= p.n_total) return;
        scatter_agent<DIM>(p, P, I, count, start, Ps, Is, i);
        return;
    }
    chem_slab_body<DIM, NS, UPT, 1>(p, q, inst, Ps, start, nullptr, nullptr, Ssrc, Supt, By, Bz,
                                    nby, nbz, 0, split, slab_cnt, slab_tab, flags,
                                    (int)(blockIdx.x - nsc));
}

// After k_slab_classify: the first nslabs work-groups deposit (and update)
// the light slabs, the rest assist with the heavy slabs' chunks, so that
// both kinds of work run side by side in one grid.
template <int DIM, int NS, bool UPT>
__global__ void __launch_bounds__(kSlabThreads)
k_slab_merged(StepParams p, PdeParams q, const InstInfo *__restrict__ inst,
              const float4 *__restrict__ Ps, const uint32_t *__restrict__ start,
              const float *__restrict__ cin, float *__restrict__ cout,
              unsigned long long *__restrict__ Ssrc, unsigned long long *__restrict__ Supt,
              int By, int Bz, int nby, int nbz, int fuse_pde, uint32_t split, int nslabs,
              uint32_t *__restrict__ slab_cnt, uint32_t *__restrict__ slab_tab,
              uint32_t *__restrict__ flags, uint32_t *__restrict__ stepc) {
    if (fuse_pde && stepc && blockIdx.x == 0 && threadIdx.x == 0) *stepc += 1u;
    if ((int)blockIdx.x < nslabs)
        chem_slab_body<DIM, NS, UPT, 2>(p, q, inst, Ps, start, cin, cout, Ssrc, Supt, By, Bz,
                                        nby, nbz, fuse_pde, split, slab_cnt, slab_tab, flags,
                                        (int)blockIdx.x);
    else
        slab_assist_body<DIM, NS, UPT>(p, inst, Ps, Ssrc, Supt, By, Bz, nby, nbz, nslabs,
                                       slab_cnt, slab_tab, blockIdx.x - (uint32_t)nslabs,
                                       gridDim.x - (uint32_t)nslabs);
}

// The single PDE substep at the nodes of the handed-over slabs, from their
// deposits in HBM (the other slabs applied it in k_chem_slabs), a quarter
// of a slab's nodes per work-group.
template <int DIM, bool UPT>
__global__ void __launch_bounds__(256)
k_slab_finish(StepParams p, PdeParams q, const InstInfo *__restrict__ inst,
              const float *__restrict__ cin, float *__restrict__ cout,
              const unsigned long long *__restrict__ Ssrc,
              const unsigned long long *__restrict__ Supt, int By, int Bz, int nby, int nbz,
              const uint32_t *__restrict__ slab_cnt, uint32_t *__restrict__ flags) {
    const int sl = blockIdx.x / kFinishParts, part = blockIdx.x % kFinishParts;
    if (slab_cnt[sl] == 0u) return;
    const int n = p.grid_n;
    const SlabGeom g = slab_geom<DIM>(sl, n, By, Bz, nby, nbz);
    const InstInfo ii = inst[g.k];
    const int per = (g.owned + kFinishParts - 1) / kFinishParts;
    uint32_t flag = 0;
    slab_pde_nodes<DIM, UPT, true>(q, g, ii, n, cin, cout, Ssrc, Supt, part * per,
                                   min(g.owned, (part + 1) * per), flag);
    if (flag) atomicOr(flags, flag);
}

// Slab heights (y rows By, z layers Bz) of the owner-computes deposit: about
// 2048 owned nodes (16 KB of LDS sums per field) and enough slabs to fill
// the chip.  A slab's runs are its z bin layers, one per y interval (two
// where the slab touches the periodic seam): at most 2 ((Bz + 2) f + 6) for
// f bins per cell.  Returns false when no height keeps them within
// kSlabRuns (very fine bins on a coarse grid): the step then deposits with
// device atomics.
bool chem_slab_shape(int dim, int n, double f, int n_inst, SlabShape &sh) {
    int By = 4, Bz = 1;
    if (dim == 3) {
        Bz = 4;
        while (n * By * Bz > 2048 && (By > 1 || Bz > 1)) {
            if (By >= Bz) By /= 2;
            else Bz /= 2;
        }
        while (Bz > 1 && 2.0 * ((Bz + 2) * f + 6.0) > kSlabRuns - 1) Bz /= 2;
        if (2.0 * ((Bz + 2) * f + 6.0) > kSlabRuns - 1) return false;
    } else {
        while (n * By > 2048 && By > 1) By /= 2;
    }
    sh.By = By;
    sh.Bz = Bz;
    sh.nby = (n + By - 1) / By;
    sh.nbz = dim == 3 ? (n + Bz - 1) / Bz : 1;
    sh.nslabs = (int64_t)sh.nby * sh.nbz * n_inst;
    sh.lds_bytes = 8 * (size_t)n * By * Bz;   // per deposited field
    sh.assist_blocks = kAssistBlocks;
    return true;
}

// One round of resident work-groups takes every chunk of the handed-over
// slabs at once where they number fewer (the 1M-agent 3D run has about
// 1,400 chunks): on 256 CUs with six resident work-groups each, 1536
// work-groups instead of 1024 cut the assist by ~2 us per step, while a
// second round (2048) or more than fit (1792) made it slower.
template <int DIM, int NS, bool UPT>
static int assist_occupancy(size_t lds) {
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &occ, reinterpret_cast<const void *>(&k_slab_assist<DIM, NS, UPT>), kAssistThreads,
            lds) != hipSuccess)
        return 0;
    return occ;
}

void chem_slab_assist_grid(const StepParams &p, SlabShape &sh) {
    const bool upt = p.has_uptake != 0;
    const size_t lds = sh.lds_bytes * (upt ? 2 : 1);
    const int ns = p.n_species == 1 ? 1 : (p.n_species == 2 ? 2 : 0);
    int occ = 0;
#define PC_OCC(D, N) occ = upt ? assist_occupancy<D, N, true>(lds) : assist_occupancy<D, N, false>(lds)
    if (p.dim == 2) {
        if (ns == 1) PC_OCC(2, 1);
        else if (ns == 2) PC_OCC(2, 2);
        else PC_OCC(2, 0);
    } else {
        if (ns == 1) PC_OCC(3, 1);
        else if (ns == 2) PC_OCC(3, 2);
        else PC_OCC(3, 0);
    }
#undef PC_OCC
    int dev = 0, cus = 0;
    if (occ <= 0 || hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0) {
        (void)hipGetLastError();
        sh.assist_blocks = kAssistBlocks;
        return;
    }
    sh.assist_blocks = occ * cus;
}

size_t chem_slab_table_words() { return kSlabTableWords; }

template <int DIM, int NS, bool UPT>
static void slabs(const StepParams &p, const PdeParams &q, const Buffers &b, const SlabShape &sh,
                  uint32_t split, int src, int cur, int fuse, int classify, hipStream_t s) {
    const size_t lds = sh.lds_bytes * (UPT ? 2 : 1);
    if (classify)
        hipLaunchKernelGGL((k_slab_classify<DIM, NS, UPT>), dim3((unsigned)sh.nslabs),
                           dim3(kSlabThreads), 0, s, p, q, b.inst, b.P[src], b.start, b.S_src,
                           b.S_upt, sh.By, sh.Bz, sh.nby, sh.nbz, split, b.slab_cnt,
                           b.slab_tab, b.flags);
    hipLaunchKernelGGL((k_slab_merged<DIM, NS, UPT>),
                       dim3((unsigned)(sh.nslabs + sh.assist_blocks)), dim3(kSlabThreads), lds,
                       s, p, q, b.inst, b.P[src], b.start, b.c[cur], b.c[1 - cur], b.S_src,
                       b.S_upt, sh.By, sh.Bz, sh.nby, sh.nbz, fuse, split, (int)sh.nslabs,
                       b.slab_cnt, b.slab_tab, b.flags, b.step);
    if (fuse)
        hipLaunchKernelGGL((k_slab_finish<DIM, UPT>), dim3((unsigned)(sh.nslabs * kFinishParts)),
                           dim3(256), 0, s,
                           p, q, b.inst, b.c[cur], b.c[1 - cur], b.S_src, b.S_upt, sh.By, sh.Bz,
                           sh.nby, sh.nbz, b.slab_cnt, b.flags);
}

void launch_chem_slabs(const StepParams &p, const PdeParams &q, const Buffers &b,
                       const SlabShape &sh, uint32_t split, int src, int cur, int fuse_pde,
                       hipStream_t s, int classify) {
    const int ns = p.n_species == 1 ? 1 : (p.n_species == 2 ? 2 : 0);
#define PC_SLAB(D, N)                                                                      \
    do {                                                                                   \
        if (p.has_uptake)                                                                  \
            slabs<D, N, true>(p, q, b, sh, split, src, cur, fuse_pde, classify, s);        \
        else                                                                               \
            slabs<D, N, false>(p, q, b, sh, split, src, cur, fuse_pde, classify, s);       \
    } while (0)
    if (p.dim == 2) {
        if (ns == 1) PC_SLAB(2, 1);
        else if (ns == 2) PC_SLAB(2, 2);
        else PC_SLAB(2, 0);
    } else {
        if (ns == 1) PC_SLAB(3, 1);
        else if (ns == 2) PC_SLAB(3, 2);
        else PC_SLAB(3, 0);
    }
#undef PC_SLAB
}


template <int DIM, int NS, bool UPT>
static void scat_cls(const StepParams &p, const PdeParams &q, const Buffers &b,
                     const SlabShape &sh, uint32_t split, int src, int dst, hipStream_t s) {
    const uint32_t nsc = (uint32_t)(((int64_t)p.n_total + kSlabThreads - 1) / kSlabThreads);
    hipLaunchKernelGGL((k_scatter_classify<DIM, NS, UPT>), dim3((unsigned)(nsc + sh.nslabs)),
                       dim3(kSlabThreads), 0, s, p, q, b.inst, b.P[src], b.I[src], b.count,
                       b.start, b.P[dst], b.I[dst], b.S_src, b.S_upt, sh.By, sh.Bz, sh.nby,
                       sh.nbz, split, b.slab_cnt, b.slab_tab, b.flags, nsc);
}

void launch_scatter_classify(const StepParams &p, const PdeParams &q, const Buffers &b,
                             const SlabShape &sh, uint32_t split, int src, int dst,
                             hipStream_t s) {
    const int ns = p.n_species == 1 ? 1 : (p.n_species == 2 ? 2 : 0);
#define PC_SC(D, N)                                                                  \
    do {                                                                             \
        if (p.has_uptake) scat_cls<D, N, true>(p, q, b, sh, split, src, dst, s);     \
        else scat_cls<D, N, false>(p, q, b, sh, split, src, dst, s);                 \
    } while (0)
    if (p.dim == 2) {
        if (ns == 1) PC_SC(2, 1);
        else if (ns == 2) PC_SC(2, 2);
        else PC_SC(2, 0);
    } else {
        if (ns == 1) PC_SC(3, 1);
        else if (ns == 2) PC_SC(3, 2);
        else PC_SC(3, 0);
    }
#undef PC_SC
}

}  // namespace pc
