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
#include "pc_internal.h"

namespace pc {

// ---------------------------------------------------------------------------
// Launch helpers
// ---------------------------------------------------------------------------

// Work-groups are dealt to the 8 XCDs round robin.  Give each XCD one
// contiguous chunk of logical blocks, so that spatially adjacent agents
// (adjacent in cell-sorted order) share an XCD's L2.
__device__ __forceinline__ uint32_t xcd_block(uint32_t bid, uint32_t nblocks) {
    const uint32_t nx = 8;
    const uint32_t per = nblocks / nx, rem = nblocks % nx;
    const uint32_t x = bid % nx, k = bid / nx;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + k;
}

__device__ __forceinline__ uint32_t inst_of(float w) { return __float_as_uint(w) >> 8; }
__device__ __forceinline__ int species_of(float w) { return (int)(__float_as_uint(w) & 0xffu); }

// ---------------------------------------------------------------------------
// Counter-based noise: Philox4x32-10 (Salmon, Moraes, Dror & Shaw, SC'11).
// ---------------------------------------------------------------------------
struct U4 { uint32_t v[4]; };

__device__ __forceinline__ U4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
        const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
        const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += W0; k1 += W1;
    }
    U4 o;
    o.v[0] = c0; o.v[1] = c1; o.v[2] = c2; o.v[3] = c3;
    return o;
}

// Uniform in (0,1): top 24 bits with the last kept bit set, times 2^-24.
__device__ __forceinline__ float uniform24(uint32_t w) {
    return (float)((w >> 8) | 1u) * 5.9604644775390625e-8f;
}

// Box-Muller normals: (xi0, xi1) from words 0, 1 and xi2 from words 2, 3.
template <int DIM>
__device__ __forceinline__ void normals(const U4 &w, float xi[3]) {
    const float u0 = uniform24(w.v[0]), u1 = uniform24(w.v[1]);
    const float r0 = sqrtf(-2.0f * logf(u0));
    float s1, c1;
    sincospif(2.0f * u1, &s1, &c1);
    xi[0] = r0 * c1;
    xi[1] = r0 * s1;
    xi[2] = 0.0f;
    if (DIM == 3) {
        const float u2 = uniform24(w.v[2]), u3 = uniform24(w.v[3]);
        const float r1 = sqrtf(-2.0f * logf(u2));
        xi[2] = r1 * cospif(2.0f * u3);
    }
}

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
    unsigned long long z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// ---------------------------------------------------------------------------
// Species tables: NS = 1 or 2 select from registers, otherwise LDS.
// ---------------------------------------------------------------------------
struct SpTab {
    float cut2[kMaxSpecies * kMaxSpecies];
    float dij[kMaxSpecies * kMaxSpecies];
    float amp[kMaxSpecies], chi[kMaxSpecies], src[kMaxSpecies], upt[kMaxSpecies];
};

__device__ __forceinline__ void load_tab(const StepParams &p, SpTab &t) {
    const int n2 = p.n_species * p.n_species;
    for (int q = threadIdx.x; q < n2; q += blockDim.x) {
        t.cut2[q] = p.cut2[q];
        t.dij[q] = p.dij[q];
    }
    for (int q = threadIdx.x; q < p.n_species; q += blockDim.x) {
        t.amp[q] = p.amp[q];
        t.chi[q] = p.chi[q];
        t.src[q] = p.src_fx[q];
        t.upt[q] = p.upt_fx[q];
    }
}

template <int NS>
__device__ __forceinline__ float sel(const float *kern, const float *lds, int s) {
    if (NS == 1) return kern[0];
    if (NS == 2) return s ? kern[1] : kern[0];
    return lds[s];
}

// ---------------------------------------------------------------------------
// Cell-list bins.  nb bins per axis of side L / nb; global bin =
// instance bin base + bx + nb (by + nb bz).
// ---------------------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ uint32_t agent_bin(const StepParams &p, float4 x) {
    const float top = (float)(p.nb - 1);
    const int bx = (int)fminf(fmaxf(x.x * p.inv_bin, 0.0f), top);
    const int by = (int)fminf(fmaxf(x.y * p.inv_bin, 0.0f), top);
    int bz = 0;
    if (DIM == 3) bz = (int)fminf(fmaxf(x.z * p.inv_bin, 0.0f), top);
    return (uint32_t)(bx + p.nb * (by + p.nb * bz));
}

// Pair loop over the neighbour bins of agent `self` (cell-sorted index) at
// position pi.  Accumulates the repulsion F_i = -sum k (d_ij - r) dx / r
// over neighbours with r > 0 and, in debug mode, the neighbour count and id
// hash.  dx = x_j - x_i, plus -L / +L for bins reached through the periodic
// seam: for every pair closer than the cutoff this is exactly the minimum
// image, because the seam is crossed iff |x_j - x_i| > L/2 for such pairs.
template <int DIM, int NS, int STENCIL, bool DBG>
__device__ __forceinline__ void pair_loop(const StepParams &p, const SpTab &tab,
                                          const float4 *__restrict__ Ps,
                                          const uint32_t *__restrict__ Is,
                                          const uint32_t *__restrict__ start, uint32_t bin_base,
                                          uint32_t self, float4 pi, int si, float F[3],
                                          uint32_t &cnt, unsigned long long &hsum) {
    const int nb = p.nb;
    const float pc[3] = {pi.x, pi.y, pi.z};
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const float s = fmaxf(pc[a] * p.inv_bin, 0.0f);
        const int b = min((int)s, nb - 1);
        if (STENCIL == 3) {
            lo[a] = b - 1;
            hi[a] = b + 1;
        } else {
            const int up = (s - (float)b) >= 0.5f ? 1 : 0;
            lo[a] = b - 1 + up;
            hi[a] = lo[a] + 1;
        }
    }
    // contact tables of species si
    float c2row[2] = {0.f, 0.f}, drow[2] = {0.f, 0.f};
    if (NS == 1) {
        c2row[0] = p.cut2[0];
        drow[0] = p.dij[0];
    } else if (NS == 2) {
        c2row[0] = p.cut2[si * 2 + 0];
        c2row[1] = p.cut2[si * 2 + 1];
        drow[0] = p.dij[si * 2 + 0];
        drow[1] = p.dij[si * 2 + 1];
    }
    const float L = p.L;
    const float kk = p.k;

    auto scan = [&](uint32_t a, uint32_t e, float sx, float sy, float sz) {
        for (uint32_t j = a; j < e; ++j) {
            const float4 q = Ps[j];
            const float dx = (q.x - pi.x) + sx;
            const float dy = (q.y - pi.y) + sy;
            float r2 = dx * dx + dy * dy;
            float dz = 0.0f;
            if (DIM == 3) {
                dz = (q.z - pi.z) + sz;
                r2 = r2 + dz * dz;
            }
            float c2, dd;
            if (NS == 1) {
                c2 = c2row[0];
                dd = drow[0];
            } else if (NS == 2) {
                const int sj = species_of(q.w);
                c2 = sj ? c2row[1] : c2row[0];
                dd = sj ? drow[1] : drow[0];
            } else {
                const int sj = species_of(q.w);
                c2 = tab.cut2[si * p.n_species + sj];
                dd = tab.dij[si * p.n_species + sj];
            }
            if (r2 < c2 && j != self) {
                if (DBG) {
                    cnt += 1;
                    hsum += splitmix64((unsigned long long)Is[j]);
                }
                if (r2 > 0.0f) {
                    const float r = sqrtf(r2);
                    const float f = kk * (dd - r) / r;
                    F[0] -= f * dx;
                    F[1] -= f * dy;
                    if (DIM == 3) F[2] -= f * dz;
                }
            }
        }
    };

    const int zlo = DIM == 3 ? lo[2] : 0, zhi = DIM == 3 ? hi[2] : 0;
    for (int oz = zlo; oz <= zhi; ++oz) {
        int qz = oz;
        float sz = 0.0f;
        if (DIM == 3) {
            if (qz < 0) {
                if (!p.periodic) continue;
                qz += nb;
                sz = -L;
            } else if (qz >= nb) {
                if (!p.periodic) continue;
                qz -= nb;
                sz = L;
            }
        }
        for (int oy = lo[1]; oy <= hi[1]; ++oy) {
            int qy = oy;
            float sy = 0.0f;
            if (qy < 0) {
                if (!p.periodic) continue;
                qy += nb;
                sy = -L;
            } else if (qy >= nb) {
                if (!p.periodic) continue;
                qy -= nb;
                sy = L;
            }
            const uint32_t row = bin_base + (uint32_t)((qz * nb + qy) * nb);
            const int m0 = max(lo[0], 0), m1 = min(hi[0], nb - 1);
            scan(start[row + m0], start[row + m1 + 1], 0.0f, sy, sz);
            if (p.periodic) {
                if (lo[0] < 0) scan(start[row + lo[0] + nb], start[row + nb], -L, sy, sz);
                if (hi[0] > nb - 1) scan(start[row], start[row + hi[0] - nb + 1], L, sy, sz);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Grid geometry.  Periodic: spacing L/n, nodes i*h, upper corner wraps.
// Walls: spacing L/(n-1), nodes on both walls, lower corner <= n-2.
// ---------------------------------------------------------------------------
struct Cell { int i0, i1; float t; };

__device__ __forceinline__ Cell cell_of(const StepParams &p, float x) {
    const float s = fmaxf(x * p.inv_h, 0.0f);
    const float fi = fminf(floorf(s), p.cell_top);
    Cell c;
    c.i0 = (int)fi;
    c.t = s - fi;
    c.i1 = c.i0 + 1;
    if (p.periodic && c.i1 == p.grid_n) c.i1 = 0;
    return c;
}

// index at offset -1 / +2 of a cell's lower corner, periodic wrap or mirror
__device__ __forceinline__ int idx_m1(const StepParams &p, int i0) {
    if (i0 > 0) return i0 - 1;
    return p.periodic ? p.grid_n - 1 : 1;
}
__device__ __forceinline__ int idx_p2(const StepParams &p, int i0) {
    const int q = i0 + 2;
    if (q < p.grid_n) return q;
    return p.periodic ? q - p.grid_n : p.grid_n - 2;
}

// Multilinear interpolation at x of the centred-difference gradient of c,
// computed on the fly from the 4^dim-minus-corners stencil of c around the
// agent's cell (the node gradient field itself is never stored).
template <int DIM>
__device__ __forceinline__ void grad_interp(const StepParams &p, const float *__restrict__ c,
                                            float4 x, float g[3]) {
    const Cell cx = cell_of(p, x.x), cy = cell_of(p, x.y);
    const int n = p.grid_n;
    const int X4[4] = {idx_m1(p, cx.i0), cx.i0, cx.i1, idx_p2(p, cx.i0)};
    const int Y4[4] = {idx_m1(p, cy.i0), cy.i0, cy.i1, idx_p2(p, cy.i0)};
    const float wx[2] = {1.0f - cx.t, cx.t}, wy[2] = {1.0f - cy.t, cy.t};
    const float ih2 = p.inv_2h;
    if (DIM == 2) {
        float gx = 0.f, gy = 0.f;
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                const int ry = Y4[b + 1] * n, rx = X4[a + 1];
                const float ddx = c[ry + X4[a + 2]] - c[ry + X4[a]];
                const float ddy = c[Y4[b + 2] * n + rx] - c[Y4[b] * n + rx];
                const float w = wx[a] * wy[b];
                gx = fmaf(w, ddx, gx);
                gy = fmaf(w, ddy, gy);
            }
        g[0] = gx * ih2;
        g[1] = gy * ih2;
        g[2] = 0.f;
    } else {
        const Cell cz = cell_of(p, x.z);
        const int Z4[4] = {idx_m1(p, cz.i0), cz.i0, cz.i1, idx_p2(p, cz.i0)};
        const float wz[2] = {1.0f - cz.t, cz.t};
        const int nn = n * n;
        float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const int zo = Z4[e + 1] * nn, yo = Y4[b + 1] * n, xo = X4[a + 1];
                    const float ddx = c[zo + yo + X4[a + 2]] - c[zo + yo + X4[a]];
                    const float ddy = c[zo + Y4[b + 2] * n + xo] - c[zo + Y4[b] * n + xo];
                    const float ddz = c[Z4[e + 2] * nn + yo + xo] - c[Z4[e] * nn + yo + xo];
                    const float w = wx[a] * wy[b] * wz[e];
                    gx = fmaf(w, ddx, gx);
                    gy = fmaf(w, ddy, gy);
                    gz = fmaf(w, ddz, gz);
                }
        g[0] = gx * ih2;
        g[1] = gy * ih2;
        g[2] = gz * ih2;
    }
}

// Piecewise-linear deposit of q (fixed point) at x into S.
template <int DIM>
__device__ __forceinline__ void deposit(const StepParams &p, unsigned long long *__restrict__ S,
                                        float q, const Cell *cc) {
    const int n = p.grid_n;
#pragma unroll
    for (int m = 0; m < (1 << DIM); ++m) {
        float w = q;
        int idx = 0, stride = 1;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int up = (m >> a) & 1;
            w *= up ? cc[a].t : 1.0f - cc[a].t;
            idx += (up ? cc[a].i1 : cc[a].i0) * stride;
            stride *= n;
        }
        const unsigned long long v = (unsigned long long)__float2ull_rn(w);
        if (v) atomicAdd(S + idx, v);
    }
}

__device__ __forceinline__ float boundary(const StepParams &p, float x, uint32_t &flag) {
    const float L = p.L;
    if (p.periodic) {
        x = x - L * floorf(x / L);
        if (x >= L) x -= L;
        if (!(x >= 0.0f)) {
            x = 0.0f;
            flag |= FLAG_WARN_CLAMPED;
        }
        return x;
    }
    if (x < 0.0f) x = -x;
    else if (x > L) x = 2.0f * L - x;
    if (x < 0.0f || x > L) {
        x = fminf(fmaxf(x, 0.0f), L);
        flag |= FLAG_WARN_CLAMPED;
    }
    return x;
}

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

template <int DIM>
__global__ void k_bin(StepParams p, const InstInfo *__restrict__ inst,
                      const float4 *__restrict__ P, uint32_t *__restrict__ bin,
                      uint32_t *__restrict__ rank, uint32_t *__restrict__ count) {
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int i = blk * blockDim.x + threadIdx.x;
    if (i >= p.n_total) return;
    const float4 x = P[i];
    const uint32_t b = inst[inst_of(x.w)].bin_base + agent_bin<DIM>(p, x);
    bin[i] = b;
    rank[i] = atomicAdd(count + b, 1u);
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

__global__ void __launch_bounds__(256) k_tile_sums(const uint32_t *__restrict__ count,
                                                   int64_t n, uint32_t *__restrict__ tile_sum) {
    __shared__ uint32_t lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (base + k < n) s += count[base + k];
    uint32_t tot;
    block_exscan256(s, lds, tot);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(1024) k_scan_tiles(uint32_t *__restrict__ tile_sum, int T) {
    __shared__ uint32_t lds[16];
    const int per = (T + 1023) / 1024;
    const int b0 = threadIdx.x * per;
    uint32_t s = 0;
    for (int k = 0; k < per; ++k)
        if (b0 + k < T) s += tile_sum[b0 + k];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t x = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) lds[wv] = x;
    __syncthreads();
    uint32_t base = 0;
    for (int k = 0; k < wv; ++k) base += lds[k];
    uint32_t run = base + x - s;
    for (int k = 0; k < per; ++k)
        if (b0 + k < T) {
            const uint32_t t = tile_sum[b0 + k];
            tile_sum[b0 + k] = run;
            run += t;
        }
}

__global__ void __launch_bounds__(256) k_scan_apply(uint32_t *__restrict__ count, int64_t n,
                                                    const uint32_t *__restrict__ tile_sum,
                                                    uint32_t *__restrict__ start) {
    __shared__ uint32_t lds[4];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 8;
    uint32_t v[8];
    uint32_t s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        v[k] = base + k < n ? count[base + k] : 0u;
        s += v[k];
    }
    uint32_t tot;
    uint32_t run = block_exscan256(s, lds, tot) + tile_sum[blockIdx.x];
#pragma unroll
    for (int k = 0; k < 8; ++k)
        if (base + k < n) {
            start[base + k] = run;
            count[base + k] = 0u;
            run += v[k];
        }
}

__global__ void k_scatter(int n, const float4 *__restrict__ P, const uint32_t *__restrict__ I,
                          const uint32_t *__restrict__ bin, const uint32_t *__restrict__ rank,
                          const uint32_t *__restrict__ start, float4 *__restrict__ Ps,
                          uint32_t *__restrict__ Is) {
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int i = blk * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t d = start[bin[i]] + rank[i];
    Ps[d] = P[i];
    Is[d] = I[i];
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
// with Philox normals, boundary closure, deposit at X^{n+1}.
template <int DIM, int NS, int STENCIL>
__global__ void __launch_bounds__(1024)
k_update(StepParams p, const InstInfo *__restrict__ inst, const float4 *__restrict__ Ps,
         const uint32_t *__restrict__ Is, const uint32_t *__restrict__ start,
         const float *__restrict__ c, float4 *__restrict__ Pout, uint32_t *__restrict__ Iout,
         unsigned long long *__restrict__ Ssrc, unsigned long long *__restrict__ Supt,
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
    const uint32_t k = inst_of(pi.w);
    const InstInfo ii = inst[k];

    float F[3] = {0.f, 0.f, 0.f};
    uint32_t cnt = 0;
    unsigned long long hs = 0;
    pair_loop<DIM, NS, STENCIL, false>(p, tab, Ps, Is, start, ii.bin_base, (uint32_t)i, pi, si,
                                       F, cnt, hs);

    float drift[3] = {0.f, 0.f, 0.f};
    const float chi = sel<NS>(p.chi, tab.chi, si) * ii.chi_scale;
    if (chi != 0.0f) {
        float g[3];
        grad_interp<DIM>(p, c + ii.node_base, pi, g);
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
    xn.x = boundary(p, pi.x + p.dt * (F[0] + drift[0]) + amp * xi[0], flag);
    xn.y = boundary(p, pi.y + p.dt * (F[1] + drift[1]) + amp * xi[1], flag);
    xn.z = DIM == 3 ? boundary(p, pi.z + p.dt * (F[2] + drift[2]) + amp * xi[2], flag) : 0.0f;
    xn.w = pi.w;
    if (!(isfinite(xn.x) && isfinite(xn.y) && isfinite(xn.z))) flag |= FLAG_NONFINITE;
    Pout[i] = xn;
    Iout[i] = id;

    Cell cc[3];
    cc[0] = cell_of(p, xn.x);
    cc[1] = cell_of(p, xn.y);
    if (DIM == 3) cc[2] = cell_of(p, xn.z);
    const float qs = sel<NS>(p.src_fx, tab.src, si);
    if (qs != 0.0f) deposit<DIM>(p, Ssrc + ii.node_base, qs, cc);
    if (p.has_uptake) {
        const float qu = sel<NS>(p.upt_fx, tab.upt, si);
        if (qu != 0.0f) deposit<DIM>(p, Supt + ii.node_base, qu, cc);
    }
    if (flag) atomicOr(flags, flag);
}

// Forward-Euler substep of the chemical with the centred Laplacian (periodic
// wrap or mirror ghost nodes), fixed-point deposits converted to number
// densities with the node control volumes.  The last substep clears the
// deposits and advances the step counter.
template <int DIM>
__global__ void k_pde(PdeParams q, const float *__restrict__ cin, float *__restrict__ cout,
                      unsigned long long *__restrict__ Ssrc, unsigned long long *__restrict__ Supt,
                      int last, uint32_t *__restrict__ stepc, uint32_t *__restrict__ flags) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (last && l == 0) *stepc += 1u;
    if (l >= q.n_nodes_total) return;
    const int n = q.grid_n;
    const int64_t G = q.nodes_per_inst;
    const int64_t base = (l / G) * G;
    const int loc = (int)(l - base);
    const int ix = loc % n, iy = (loc / n) % n, iz = DIM == 3 ? loc / (n * n) : 0;
    auto nb = [&](int i, int off) {
        int r = i + off;
        if (q.periodic) return r < 0 ? r + n : (r >= n ? r - n : r);
        return r < 0 ? 1 : (r >= n ? n - 2 : r);
    };
    const float *cb = cin + base;
    const float c0 = cb[loc];
    const int nn = n * n;
    const int rowo = iz * nn + iy * n;
    float lap = (cb[rowo + nb(ix, 1)] + cb[rowo + nb(ix, -1)]) +
                (cb[iz * nn + nb(iy, 1) * n + ix] + cb[iz * nn + nb(iy, -1) * n + ix]);
    float diag = 4.0f;
    if (DIM == 3) {
        lap += cb[nb(iz, 1) * nn + iy * n + ix] + cb[nb(iz, -1) * nn + iy * n + ix];
        diag = 6.0f;
    }
    lap = (lap - diag * c0) * q.inv_h2;
    float inv_v = 1.0f;
    if (!q.periodic) {
        if (ix == 0 || ix == n - 1) inv_v *= 2.0f;
        if (iy == 0 || iy == n - 1) inv_v *= 2.0f;
        if (DIM == 3 && (iz == 0 || iz == n - 1)) inv_v *= 2.0f;
    }
    const float dens = q.fx_to_density * inv_v;
    const float sigma = (float)Ssrc[l] * dens;
    float ups = 0.0f;
    if (q.has_uptake) ups = (float)Supt[l] * dens;
    const float cn = c0 + q.dts * (q.D_c * lap + sigma - ups * c0 - q.gamma * c0);
    cout[l] = cn;
    uint32_t flag = 0;
    if (!isfinite(cn)) flag |= FLAG_NONFINITE;
    if (q.dts * (q.gamma + ups) >= 1.0f) flag |= FLAG_WARN_POSITIVITY;
    if (flag) atomicOr(flags, flag);
    if (last) {
        Ssrc[l] = 0ull;
        if (q.has_uptake) Supt[l] = 0ull;
    }
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

template <int DIM, int NS, int STENCIL>
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
    float F[3] = {0.f, 0.f, 0.f};
    uint32_t cnt = 0;
    unsigned long long hs = 0;
    pair_loop<DIM, NS, STENCIL, true>(p, tab, Ps, Is, start, ii.bin_base, (uint32_t)i, pi, si, F,
                                      cnt, hs);
    const size_t row = ii.agent_base + Is[i];
    if (count) count[row] = cnt;
    if (hash) hash[row] = hs;
    if (Fo)
        for (int a = 0; a < DIM; ++a) Fo[row * DIM + a] = F[a];
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
        hipLaunchKernelGGL(k_bin<2>, g, t, 0, s, p, b.inst, b.P[src], b.bin, b.rank, b.count);
    else
        hipLaunchKernelGGL(k_bin<3>, g, t, 0, s, p, b.inst, b.P[src], b.bin, b.rank, b.count);
}

void launch_scan(const Buffers &b, int64_t n_bins_total, int32_t n_total, hipStream_t s) {
    (void)n_total;
    const int64_t n = n_bins_total + 1;  // count[n_bins_total] is always 0
    const int T = (int)((n + kScanTile - 1) / kScanTile);
    hipLaunchKernelGGL(k_tile_sums, dim3(T), dim3(256), 0, s, b.count, n, b.tile_sum);
    hipLaunchKernelGGL(k_scan_tiles, dim3(1), dim3(1024), 0, s, b.tile_sum, T);
    hipLaunchKernelGGL(k_scan_apply, dim3(T), dim3(256), 0, s, b.count, n, b.tile_sum, b.start);
}

void launch_scatter(const StepParams &p, const Buffers &b, int src, int dst, int block,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_scatter, dim3(grid_for(p.n_total, block)), dim3(block), 0, s, p.n_total,
                       b.P[src], b.I[src], b.bin, b.rank, b.start, b.P[dst], b.I[dst]);
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

template <int DIM, int NS, int ST>
static void upd(const StepParams &p, const Buffers &b, int src, int dst, int cbuf, int block,
                hipStream_t s) {
    hipLaunchKernelGGL((k_update<DIM, NS, ST>), dim3(grid_for(p.n_total, block)), dim3(block), 0,
                       s, p, b.inst, b.P[src], b.I[src], b.start, b.c[cbuf], b.P[dst], b.I[dst],
                       b.S_src, b.S_upt, b.step, b.flags);
}

template <int DIM, int NS, int ST>
static void dbg(const StepParams &p, const Buffers &b, int src, uint32_t *count,
                unsigned long long *hash, float *F, int block, hipStream_t s) {
    hipLaunchKernelGGL((k_debug_pairs<DIM, NS, ST>), dim3(grid_for(p.n_total, block)),
                       dim3(block), 0, s, p, b.inst, b.P[src], b.I[src], b.start, count, hash, F);
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
    PC_DISPATCH(upd, p, b, src, dst, cbuf, block, s);
}

void launch_debug_pairs(const StepParams &p, const Buffers &b, int src, uint32_t *count,
                        unsigned long long *hash, float *F, int block, hipStream_t s) {
    PC_DISPATCH(dbg, p, b, src, count, hash, F, block, s);
}

void launch_pde(const PdeParams &q, const Buffers &b, int cin, int cout, int last,
                hipStream_t s) {
    const dim3 g(grid_for(q.n_nodes_total, 256)), t(256);
    if (q.dim == 2)
        hipLaunchKernelGGL(k_pde<2>, g, t, 0, s, q, b.c[cin], b.c[cout], b.S_src, b.S_upt, last,
                           b.step, b.flags);
    else
        hipLaunchKernelGGL(k_pde<3>, g, t, 0, s, q, b.c[cin], b.c[cout], b.S_src, b.S_upt, last,
                           b.step, b.flags);
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

void launch_set_u32(uint32_t *ptr, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(1), 0, s, ptr, v);
}

void launch_copy_f32(float *dst, const float *src, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_copy_f32, dim3(grid_for(n, 256)), dim3(256), 0, s, dst, src, n);
}

}  // namespace pc
