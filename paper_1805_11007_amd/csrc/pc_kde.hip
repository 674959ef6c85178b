// Gaussian kernel density deposit (Sect. 2.3; the density loop of Sect. 3.5
// gathers, for every grid node, the agents within a cutoff of it): for node
// p_l, sigma_l = sum_i source_{s_i} K_{eps_i}(p_l - X_i) and upsilon_l the
// same with uptake, K_eps(x) = (2 pi eps^2)^(-dim/2) exp(-|x|^2 / (2 eps^2)),
// eps = the agent's species diameter, over |p_l - X_i| < kde_radius * eps.
// One thread per node walks the cell-list bins that overlap the ball of the
// largest radius around it, row by row (x-adjacent bins are contiguous in
// the sorted agent array), so the gather needs no atomics and sums in a
// fixed order.  A wave takes a run of nodes along x: its lanes share one
// (y, z) node row, so they walk the same bin rows with the same culling
// (compact 4 x 4 x 4 node tiles, whose lanes differ in y and z, ran 2.2x
// slower on the 1M-agent 3D workload).  In 3D the bin rows of a node are
// dealt round robin to the S waves of a work-group (threadIdx.y), whose
// partial sums are added in LDS in the fixed order 0 .. S-1: a node inside
// a dense cluster then no longer holds one wave for its whole ball.
#include <hip/hip_runtime.h>

#include "pc_device.h"
#include "pc_kde.h"

namespace pc {

constexpr int kKdeSplit = 4;  // waves sharing one 3D node run's bin rows
constexpr int kKdeAhead = 4;  // agent loads issued ahead in the gather

template <int DIM, int S>
__global__ void __launch_bounds__(S > 1 ? 64 * S : 256)
k_kde(StepParams p, const InstInfo *__restrict__ inst, const float4 *__restrict__ Ps,
      const uint32_t *__restrict__ start, float2 *__restrict__ dens) {
    __shared__ float tR2[kMaxSpecies], tnorm[kMaxSpecies], tinv[kMaxSpecies];
    __shared__ float tsrc[kMaxSpecies], tupt[kMaxSpecies];
    __shared__ float2 part[S > 1 ? 64 * S : 1];
    if (threadIdx.y == 0 && threadIdx.x < (unsigned)p.n_species) {
        const int s = threadIdx.x;
        tR2[s] = p.kde_R2[s];
        tnorm[s] = p.kde_norm[s];
        tinv[s] = p.kde_l2e[s];
        tsrc[s] = p.src_f[s];
        tupt[s] = p.upt_f[s];
    }
    __syncthreads();
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int G = p.nodes_per_inst;
    const bool valid = l < (int64_t)G * p.n_inst;
    if (S == 1 && !valid) return;
    const int n = p.grid_n, nb = p.nb;
    const int k = valid ? (int)(l / G) : 0;
    const int loc = valid ? (int)(l - (int64_t)k * G) : 0;
    const int ic[3] = {loc % n, (loc / n) % n, DIM == 3 ? loc / (n * n) : 0};
    const float pc[3] = {ic[0] * p.h, ic[1] * p.h, DIM == 3 ? ic[2] * p.h : 0.0f};
    const uint32_t bb = inst[k].bin_base;
    // bins overlapping [p - R, p + R] on each axis
    int lo[3] = {0, 0, 0}, cnt[3] = {1, 1, 1};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        int b0 = (int)floorf((pc[a] - p.kde_R) * p.inv_bin);
        int b1 = (int)floorf((pc[a] + p.kde_R) * p.inv_bin);
        if (p.periodic) {
            cnt[a] = min(b1 - b0 + 1, nb);
            lo[a] = ((b0 % nb) + nb) % nb;
        } else {
            b0 = max(b0, 0);
            b1 = min(b1, nb - 1);
            lo[a] = b0;
            cnt[a] = b1 - b0 + 1;
        }
    }
    // distance from the node to a row of bins along y (z): zero for the
    // node's own bin row, else to the nearer face of the row's slab
    const float side = p.L / (float)nb;
    auto slab_d = [&](int a, int c) -> float {
        const float b = floorf(pc[a] * p.inv_bin);      // node's own bin (unwrapped)
        const float q = floorf((pc[a] - p.kde_R) * p.inv_bin) + (float)c;  // row's bin
        if (q < b) return pc[a] - (q + 1.0f) * side;
        if (q > b) return q * side - pc[a];
        return 0.0f;
    };
    const float R2 = p.kde_R * p.kde_R;
    float sig = 0.0f, ups = 0.0f;
    // one node-agent term, summed in the agents' sorted order
    auto eval = [&](const float4 &q) {
        float dx = pc[0] - q.x, dy = pc[1] - q.y, dz = DIM == 3 ? pc[2] - q.z : 0.0f;
        if (p.periodic) {
            dx = dx > p.halfL ? dx - p.L : (dx < -p.halfL ? dx + p.L : dx);
            dy = dy > p.halfL ? dy - p.L : (dy < -p.halfL ? dy + p.L : dy);
            if (DIM == 3) dz = dz > p.halfL ? dz - p.L : (dz < -p.halfL ? dz + p.L : dz);
        }
        float r2 = dx * dx + dy * dy;
        if (DIM == 3) r2 += dz * dz;
        const int s = species_of(q.w);
        if (r2 < tR2[s]) {
            // tinv holds log2(e) / (2 eps^2): r2 * tinv <= 6.5 at the
            // truncation radius 3 eps, in the hardware exp2's normal range
            // (1 ulp)
            const float w = tnorm[s] * __builtin_amdgcn_exp2f(-r2 * tinv[s]);
            sig = fmaf(tsrc[s], w, sig);
            ups = fmaf(tupt[s], w, ups);
        }
    };
    // bin rows (cz outer, cy inner); wave threadIdx.y takes every S-th
    const int nrows = valid ? cnt[1] * cnt[2] : 0;
    for (int rr = (int)threadIdx.y; rr < nrows; rr += S) {
        const int cz = DIM == 3 ? rr / cnt[1] : 0, cy = rr - cz * cnt[1];
        const int bz = DIM == 3 ? (lo[2] + cz) % nb : 0;
        const float dz = DIM == 3 && p.periodic ? fmaxf(slab_d(2, cz), 0.0f) : 0.0f;
        {
            const int by = (lo[1] + cy) % nb;
            const uint32_t row = bb + (uint32_t)(nb * (by + nb * bz));
            // rows beyond the ball, and x bins beyond its chord, are skipped
            // (torus only: with walls lo[] is clamped and the walk is plain)
            int x0 = lo[0], x1 = lo[0] + cnt[0];
            if (p.periodic) {
                const float dy = fmaxf(slab_d(1, cy), 0.0f);
                const float d2 = dy * dy + dz * dz;
                if (d2 >= R2) continue;
                const float ext = sqrtf(R2 - d2);
                const int c0 = (int)floorf((pc[0] - ext) * p.inv_bin);
                const int c1 = (int)floorf((pc[0] + ext) * p.inv_bin);
                const int u0 = (int)floorf((pc[0] - p.kde_R) * p.inv_bin);
                const int skip = max(c0 - u0, 0);
                x0 = lo[0] + skip;
                x1 = lo[0] + min(c1 - u0 + 1, cnt[0]);
                if (x1 <= x0) continue;
                if (x0 >= nb) {  // keep the first run's start inside the row
                    x0 -= nb;
                    x1 -= nb;
                }
            }
            const int runs = x1 > nb ? 2 : 1;
            for (int r = 0; r < runs; ++r) {
                const int a0 = r == 0 ? x0 : 0;
                const int a1 = r == 0 ? min(x1, nb) : x1 - nb;
                const uint32_t j0 = start[row + a0], j1 = start[row + a1];
                uint32_t j = j0;
                // kKdeAhead loads in flight before the first is used (a
                // lane inside a dense cluster walks thousands of agents)
                for (; j + kKdeAhead <= j1; j += kKdeAhead) {
                    float4 q[kKdeAhead];
#pragma unroll
                    for (int u = 0; u < kKdeAhead; ++u) q[u] = Ps[j + u];
#pragma unroll
                    for (int u = 0; u < kKdeAhead; ++u) eval(q[u]);
                }
                for (; j < j1; ++j) eval(Ps[j]);
            }
        }
    }
    if (S > 1) {
        part[threadIdx.y * 64 + threadIdx.x] = make_float2(sig, ups);
        __syncthreads();
        if (threadIdx.y != 0 || !valid) return;
        for (int w = 1; w < S; ++w) {
            const float2 q = part[w * 64 + threadIdx.x];
            sig += q.x;
            ups += q.y;
        }
    }
    dens[l] = make_float2(sig, ups);
}

void launch_kde(const StepParams &p, const Buffers &b, int src, hipStream_t s) {
    const int64_t total = (int64_t)p.nodes_per_inst * p.n_inst;
    float2 *dens = reinterpret_cast<float2 *>(b.S_src);
    if (p.dim == 2) {
        const dim3 g((unsigned)((total + 255) / 256)), t(256);
        hipLaunchKernelGGL((k_kde<2, 1>), g, t, 0, s, p, b.inst, b.P[src], b.start, dens);
    } else {
        // 64 nodes per work-group, their bin rows split over kKdeSplit waves
        const dim3 g((unsigned)((total + 63) / 64)), t(64, kKdeSplit);
        hipLaunchKernelGGL((k_kde<3, kKdeSplit>), g, t, 0, s, p, b.inst, b.P[src], b.start,
                           dens);
    }
}

// Agent-side deposit, one thread per cell-sorted agent (a work-group's
// agents are neighbours, so they share most nodes).  The nodes within the
// species' radius R_s of X_i have integer coordinates in
// [(X - R_s) / h, (X + R_s) / h] per axis (clamped to the grid with walls,
// wrapped on the torus, where R_s < L / 2 keeps them distinct).  Every
// agent walks the same box of nodes, so the wave stays convergent.  The
// terms source_s K and uptake_s K are summed per node in an LDS table
// (open addressing, 16 probes, then straight to the device), which is
// flushed with one device float atomic per distinct node.
constexpr int kKdeSlots = 4096;
constexpr uint32_t kKdeEmpty = 0xFFFFFFFFu;

template <int DIM>
__global__ void __launch_bounds__(1024)
k_kde_scatter(StepParams p, const InstInfo *__restrict__ inst, const float4 *__restrict__ Ps,
              float2 *__restrict__ dens) {
    __shared__ float tR2[kMaxSpecies], tnorm[kMaxSpecies], tinv[kMaxSpecies];
    __shared__ float tsrc[kMaxSpecies], tupt[kMaxSpecies];
    __shared__ uint32_t keys[kKdeSlots];
    __shared__ float vs[kKdeSlots], vu[kKdeSlots];
    if (threadIdx.x < (unsigned)p.n_species) {
        const int s = threadIdx.x;
        tR2[s] = p.kde_R2[s];
        tnorm[s] = p.kde_norm[s];
        tinv[s] = p.kde_l2e[s];
        tsrc[s] = p.src_f[s];
        tupt[s] = p.upt_f[s];
    }
    for (int q = threadIdx.x; q < kKdeSlots; q += blockDim.x) {
        keys[q] = kKdeEmpty;
        vs[q] = 0.0f;
        vu[q] = 0.0f;
    }
    __syncthreads();
    auto emit = [&](uint32_t key, float a, float b) {
        uint32_t h = (key * 2654435761u) >> 20;  // 12 bits: kKdeSlots = 4096
        for (int probe = 0; probe < 16; ++probe) {
            uint32_t old =
                __hip_atomic_load(&keys[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (old == kKdeEmpty) old = atomicCAS(&keys[h], kKdeEmpty, key);
            if (old == kKdeEmpty || old == key) {
                if (a != 0.0f) unsafeAtomicAdd(&vs[h], a);
                if (b != 0.0f) unsafeAtomicAdd(&vu[h], b);
                return;
            }
            h = (h + 1) & (kKdeSlots - 1);
        }
        if (a != 0.0f) unsafeAtomicAdd(&dens[key].x, a);
        if (b != 0.0f) unsafeAtomicAdd(&dens[key].y, b);
    };
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < p.n_total) {
        const float4 q = Ps[i];
        const int s = species_of(q.w);
        const float src = tsrc[s], upt = tupt[s];
        const float xq[3] = {q.x, q.y, q.z};
        // a non-finite position is flagged by the update; it deposits nothing
        const bool live = (src != 0.0f || upt != 0.0f) && isfinite(xq[0]) && isfinite(xq[1]) &&
                          isfinite(xq[2]);
        const int n = p.grid_n;
        // the node box is taken a hair wider than the ball (as the gather's
        // bin range), so float32 rounding of (x -+ R) / h never drops a node
        // inside it; r2 < R2 decides every node of the box
        const float R2 = tR2[s], R = sqrtf(R2) * (1.0f + 1e-4f);
        int lo[3] = {0, 0, 0}, hi[3] = {0, 0, -1};
        if (live) {
            hi[2] = 0;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                // on the torus the box stays within [-n, 2n), where one wrap
                // maps it into the grid; n nodes at most per axis
                lo[a] = max((int)ceilf((xq[a] - R) * p.inv_h), p.periodic ? -n : 0);
                hi[a] = min((int)floorf((xq[a] + R) * p.inv_h), p.periodic ? 2 * n - 1 : n - 1);
                if (hi[a] - lo[a] >= n) hi[a] = lo[a] + n - 1;
            }
        }
        const uint32_t base = inst[inst_of(q.w)].node_base;
        const float norm = tnorm[s], l2e = tinv[s];
        auto wrap = [&](int c) { return c < 0 ? c + n : (c >= n ? c - n : c); };
        for (int iz = lo[2]; iz <= hi[2]; ++iz) {
            const float dz = DIM == 3 ? (float)iz * p.h - xq[2] : 0.0f;
            const int wz = DIM == 3 ? (p.periodic ? wrap(iz) : iz) : 0;
            for (int iy = lo[1]; iy <= hi[1]; ++iy) {
                const float dy = (float)iy * p.h - xq[1];
                const int wy = p.periodic ? wrap(iy) : iy;
                const float r2yz = dy * dy + dz * dz;
                if (r2yz >= R2) continue;
                const uint32_t rowo = base + (uint32_t)((wz * n + wy) * n);
                for (int ix = lo[0]; ix <= hi[0]; ++ix) {
                    const float dx = (float)ix * p.h - xq[0];
                    const float r2 = dx * dx + r2yz;
                    if (r2 < R2) {
                        const float w = norm * __builtin_amdgcn_exp2f(-r2 * l2e);
                        emit(rowo + (uint32_t)(p.periodic ? wrap(ix) : ix), src * w, upt * w);
                    }
                }
            }
        }
    }
    __syncthreads();
    for (int q = threadIdx.x; q < kKdeSlots; q += blockDim.x) {
        const uint32_t k = keys[q];
        if (k == kKdeEmpty) continue;
        if (vs[q] != 0.0f) unsafeAtomicAdd(&dens[k].x, vs[q]);
        if (vu[q] != 0.0f) unsafeAtomicAdd(&dens[k].y, vu[q]);
    }
}

// The (sigma, upsilon) pairs start at zero: cleared at creation and by the
// last PDE substep of every step (k_pde with PdeParams::kde_clear).
void launch_kde_scatter(const StepParams &p, const Buffers &b, int src, hipStream_t s) {
    float2 *dens = reinterpret_cast<float2 *>(b.S_src);
    if (p.n_total == 0) return;
    const dim3 g((unsigned)((p.n_total + 1023) / 1024)), t(1024);
    if (p.dim == 2)
        hipLaunchKernelGGL(k_kde_scatter<2>, g, t, 0, s, p, b.inst, b.P[src], dens);
    else
        hipLaunchKernelGGL(k_kde_scatter<3>, g, t, 0, s, p, b.inst, b.P[src], dens);
}

}  // namespace pc
