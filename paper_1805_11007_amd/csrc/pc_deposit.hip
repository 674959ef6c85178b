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
// takes agents from them (consecutive threads on consecutive agents), adds
// the corners that fall in its slab into LDS sums, and then either stores
// each owned node's sums once, or, when the step has a single PDE substep,
// applies the forward-Euler update of eq. pde_c to its owned nodes
// directly (the sums never reach HBM).  Each corner is added by exactly one
// work-group, so every node receives the same integer as on every other
// deposit path (fixed point, 2^-32 units, charge times the axis weights in
// axis order), and the PDE node update is the same function as k_pde's.
#include "pc_device.h"

namespace pc {

constexpr int kSlabRuns = 256;   // contiguous agent runs per slab (LDS table)

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

template <int DIM, int NS, bool UPT>
__global__ void __launch_bounds__(1024)
k_chem_slabs(StepParams p, PdeParams q, const InstInfo *__restrict__ inst,
             const float4 *__restrict__ Ps, const uint32_t *__restrict__ start,
             const float *__restrict__ cin, float *__restrict__ cout,
             unsigned long long *__restrict__ Ssrc, unsigned long long *__restrict__ Supt,
             int By, int Bz, int nby, int nbz, int fuse_pde, uint32_t *__restrict__ flags,
             uint32_t *__restrict__ stepc) {
    extern __shared__ unsigned long long sums[];   // owned source sums, then uptake
    __shared__ uint32_t run_a[kSlabRuns];
    __shared__ uint32_t run_pre[kSlabRuns + 1];
    __shared__ uint32_t wtot[kSlabRuns / 64];
    __shared__ SpTab tab;
    // the step's last kernel advances the step counter (the update, which
    // reads it, has finished)
    if (fuse_pde && stepc && blockIdx.x == 0 && threadIdx.x == 0) *stepc += 1u;
    const int n = p.grid_n;
    const int nb = p.nb;
    const int per_inst = nby * nbz;
    const int k = blockIdx.x / per_inst;
    const int bl = blockIdx.x - k * per_inst;
    const int jy = bl % nby, jz = bl / nby;
    const int y0 = jy * By, y1 = min(y0 + By, n);
    const int z0 = DIM == 3 ? jz * Bz : 0, z1 = DIM == 3 ? min(z0 + Bz, n) : 1;
    const int owned = n * (y1 - y0) * (z1 - z0);
    const InstInfo ii = inst[k];
    for (int l = threadIdx.x; l < owned * (UPT ? 2 : 1); l += blockDim.x) sums[l] = 0ull;
    if (NS == 0) load_tab(p, tab);
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
    // agents of the runs, laid end to end; a thread's positions increase, so
    // its run index only moves forward
    int r = 0;
    for (uint32_t w = threadIdx.x; w < total; w += blockDim.x) {
        while (r + 1 < nrun && run_pre[r + 1] <= w) ++r;
        const float4 x = Ps[run_a[r] + (w - run_pre[r])];
        const int s = species_of(x.w);
        const float qs = sel<NS>(p.src_fx, tab.src, s);
        const float qu = UPT ? sel<NS>(p.upt_fx, tab.upt, s) : 0.0f;
        if (qs == 0.0f && qu == 0.0f) continue;
        Cell cc[3];
        cc[0] = cell_of(p, x.x);
        cc[1] = cell_of(p, x.y);
        cc[2] = Cell{0, 0, 0.0f};
        if (DIM == 3) cc[2] = cell_of(p, x.z);
        // owned corner offsets along y and z (-1: outside the slab)
        const int ly0 = cc[1].i0 - y0, ly1 = cc[1].i1 - y0;
        const int oy[2] = {(ly0 >= 0 && ly0 < y1 - y0) ? ly0 : -1,
                           (ly1 >= 0 && ly1 < y1 - y0) ? ly1 : -1};
        int oz[2] = {0, -1};
        if (DIM == 3) {
            const int lz0 = cc[2].i0 - z0, lz1 = cc[2].i1 - z0;
            oz[0] = (lz0 >= 0 && lz0 < z1 - z0) ? lz0 : -1;
            oz[1] = (lz1 >= 0 && lz1 < z1 - z0) ? lz1 : -1;
        }
        const int ox[2] = {cc[0].i0, cc[0].i1};
        const int ny = y1 - y0;
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
            if (oy[uy] < 0 || oz[uz] < 0) continue;
            const int l = ox[ux] + n * (oy[uy] + ny * oz[uz]);
            const unsigned long long vs = (unsigned long long)__float2ull_rn(ws);
            if (vs) atomicAdd(&sums[l], vs);
            if (UPT) {
                const unsigned long long vu = (unsigned long long)__float2ull_rn(wu);
                if (vu) atomicAdd(&sums[owned + l], vu);
            }
        }
    }
    __syncthreads();
    const int ny = y1 - y0;
    uint32_t flag = 0;
    for (int l = threadIdx.x; l < owned; l += blockDim.x) {
        const int ix = l % n, iy = y0 + (l / n) % ny, iz = z0 + l / (n * ny);
        const int64_t node = (int64_t)ii.node_base + ix + (int64_t)n * (iy + (int64_t)n * iz);
        const unsigned long long sS = sums[l], sU = UPT ? sums[owned + l] : 0ull;
        if (fuse_pde) {
            const int ic[3] = {ix, iy, iz};
            cout[node] = pde_node<DIM>(q, cin + ii.node_base, ic, sS, sU, flag);
        } else {
            Ssrc[node] = sS;
            if (UPT) Supt[node] = sU;
        }
    }
    if (flag) atomicOr(flags, flag);
}

// Slab heights (y rows By, z layers Bz) of the owner-computes deposit: about
// 2048 owned nodes (16 KB of LDS sums per field) and enough slabs to fill
// the chip.  A slab's runs are its z bin layers, one per y interval (two
// where the slab touches the periodic seam): at most 2 ((Bz + 2) f + 6) for
// f bins per cell.  Returns false when no height keeps them within
// kSlabRuns (very fine bins on a coarse grid): the step then deposits with
// device atomics.
bool chem_slab_shape(const StepParams &p, int &By, int &Bz, int &nby, int &nbz) {
    const int n = p.grid_n;
    const double f = (double)p.h * (double)p.inv_bin;
    if (p.dim == 3) {
        By = 4;
        Bz = 4;
        while (n * By * Bz > 2048 && (By > 1 || Bz > 1)) {
            if (By >= Bz) By /= 2;
            else Bz /= 2;
        }
        while (Bz > 1 && 2.0 * ((Bz + 2) * f + 6.0) > kSlabRuns - 1) Bz /= 2;
        if (2.0 * ((Bz + 2) * f + 6.0) > kSlabRuns - 1) return false;
    } else {
        By = 4;
        while (n * By > 2048 && By > 1) By /= 2;
        Bz = 1;
    }
    nby = (n + By - 1) / By;
    nbz = p.dim == 3 ? (n + Bz - 1) / Bz : 1;
    return true;
}

// LDS sums of a slab (0 when the slab path does not apply).
size_t chem_slab_lds_bytes(const StepParams &p) {
    int By, Bz, nby, nbz;
    if (!chem_slab_shape(p, By, Bz, nby, nbz)) return 0;
    return 8 * (size_t)p.grid_n * By * (p.dim == 3 ? Bz : 1) * (p.has_uptake ? 2 : 1);
}

template <int DIM, int NS, bool UPT>
static void slabs(const StepParams &p, const PdeParams &q, const Buffers &b, int src, int cur,
                  int fuse, hipStream_t s) {
    int By, Bz, nby, nbz;
    if (!chem_slab_shape(p, By, Bz, nby, nbz)) return;   // the host checked
    const size_t lds = chem_slab_lds_bytes(p);
    hipLaunchKernelGGL((k_chem_slabs<DIM, NS, UPT>), dim3((unsigned)(nby * nbz * p.n_inst)),
                       dim3(1024), lds, s, p, q, b.inst, b.P[src], b.start, b.c[cur],
                       b.c[1 - cur], b.S_src, b.S_upt, By, Bz, nby, nbz, fuse, b.flags, b.step);
}

void launch_chem_slabs(const StepParams &p, const PdeParams &q, const Buffers &b, int src,
                       int cur, int fuse_pde, hipStream_t s) {
    const int ns = p.n_species == 1 ? 1 : (p.n_species == 2 ? 2 : 0);
#define PC_SLAB(D, N)                                                    \
    do {                                                                 \
        if (p.has_uptake) slabs<D, N, true>(p, q, b, src, cur, fuse_pde, s); \
        else slabs<D, N, false>(p, q, b, src, cur, fuse_pde, s);         \
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

}  // namespace pc
