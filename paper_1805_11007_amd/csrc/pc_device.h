// Device-side building blocks shared by the step kernels (pc_kernels.hip)
// and the reverse-mode kernels (pc_adjoint.hip): block mapping, Philox
// noise, species tables, cell-list bins and pair loop, grid geometry,
// gradient interpolation and the boundary map.
#pragma once

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
        // each 32 x 32 -> 64-bit product in one multiply-add instruction
        const uint64_t p0 = (uint64_t)M0 * c0, p1 = (uint64_t)M1 * c2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
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

// Box-Muller normals: (xi0, xi1) from words 0, 1 and xi2 from words 2, 3,
// xi = sqrt(-2 ln u) (cos 2 pi v, sin 2 pi v), with the hardware base-2
// logarithm (u >= 2^-24 is a normal float), square root, sine and cosine
// (the last two take their argument in revolutions, so 2 pi v needs no
// range reduction), each within a few float32 ulps.
__device__ __forceinline__ float bm_radius(float u) {
    return __builtin_amdgcn_sqrtf(-1.38629436111989061f * __builtin_amdgcn_logf(u));
}

template <int DIM>
__device__ __forceinline__ void normals(const U4 &w, float xi[3]) {
    const float u0 = uniform24(w.v[0]), u1 = uniform24(w.v[1]);
    const float r0 = bm_radius(u0);
    xi[0] = r0 * __builtin_amdgcn_cosf(u1);
    xi[1] = r0 * __builtin_amdgcn_sinf(u1);
    xi[2] = 0.0f;
    if (DIM == 3) {
        const float u2 = uniform24(w.v[2]), u3 = uniform24(w.v[3]);
        xi[2] = bm_radius(u2) * __builtin_amdgcn_cosf(u3);
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
    float share[kMaxSpecies * kMaxSpecies];
    float amp[kMaxSpecies], chi[kMaxSpecies], src[kMaxSpecies], upt[kMaxSpecies];
};

__device__ __forceinline__ void load_tab(const StepParams &p, SpTab &t) {
    const int n2 = p.n_species * p.n_species;
    for (int q = threadIdx.x; q < n2; q += blockDim.x) {
        t.cut2[q] = p.cut2[q];
        t.dij[q] = p.dij[q];
        t.share[q] = p.hs_share[q];
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

// One candidate j.  dx = (x_j - x_i) (+ seam shift) and r2 = fma(dz, dz,
// fma(dy, dy, dx * dx)) in float32 (each fused multiply-add rounded once);
// the visitor receives every candidate with its squared contact distance c2
// and contact distance dd and decides what a neighbour is (r2 < c2).
template <int DIM, int NS, bool SHIFT, class V>
__device__ __forceinline__ void pair_one(const StepParams &p, const SpTab &tab, uint32_t j,
                                         const float4 &q, const float4 &pi, int si, float sx,
                                         float sy, float sz, const float c2row[2],
                                         const float drow[2], V &v) {
    float dx = q.x - pi.x, dy = q.y - pi.y, dz = 0.0f;
    if (SHIFT) {
        dx = dx + sx;
        dy = dy + sy;
    }
    float r2 = fmaf(dy, dy, dx * dx);
    if (DIM == 3) {
        dz = q.z - pi.z;
        if (SHIFT) dz = dz + sz;
        r2 = fmaf(dz, dz, r2);
    }
    float c2, dd;
    int sj;
    if (NS == 1) {
        c2 = c2row[0];
        dd = drow[0];
        sj = 0;
    } else if (NS == 2) {
        const bool s1 = species_of(q.w) != 0;
        c2 = s1 ? c2row[1] : c2row[0];
        dd = s1 ? drow[1] : drow[0];
        sj = s1 ? 1 : 0;
    } else {
        sj = species_of(q.w);
        c2 = tab.cut2[si * p.n_species + sj];
        dd = tab.dij[si * p.n_species + sj];
    }
    v(j, dx, dy, dz, r2, c2, dd, sj);
}

// Candidates j in [a, e) of one contiguous bin range, each as pair_one.
// Loads are issued DEEP (8: eight, then four; 4: four) candidates ahead of
// the arithmetic so that one wave keeps several memory requests in flight.
template <int DIM, int NS, bool SHIFT, class V, int DEEP = 8>
__device__ __forceinline__ void pair_range(const StepParams &p, const SpTab &tab,
                                           const float4 *__restrict__ Ps, uint32_t a,
                                           uint32_t e, const float4 &pi, int si, float sx,
                                           float sy, float sz, const float c2row[2],
                                           const float drow[2], V &v) {
    uint32_t j = a;
    // one 64-bit address per group of four; the rest are immediate offsets
    const float4 *__restrict__ qp = Ps + a;
    for (; DEEP >= 8 && j + 8 <= e; j += 8, qp += 8) {
        const float4 q0 = qp[0], q1 = qp[1], q2 = qp[2], q3 = qp[3];
        const float4 q4 = qp[4], q5 = qp[5], q6 = qp[6], q7 = qp[7];
        pair_one<DIM, NS, SHIFT>(p, tab, j, q0, pi, si, sx, sy, sz, c2row, drow, v);
        pair_one<DIM, NS, SHIFT>(p, tab, j + 1, q1, pi, si, sx, sy, sz, c2row, drow, v);
        pair_one<DIM, NS, SHIFT>(p, tab, j + 2, q2, pi, si, sx, sy, sz, c2row, drow, v);
        pair_one<DIM, NS, SHIFT>(p, tab, j + 3, q3, pi, si, sx, sy, sz, c2row, drow, v);
        pair_one<DIM, NS, SHIFT>(p, tab, j + 4, q4, pi, si, sx, sy, sz, c2row, drow, v);
        pair_one<DIM, NS, SHIFT>(p, tab, j + 5, q5, pi, si, sx, sy, sz, c2row, drow, v);
        pair_one<DIM, NS, SHIFT>(p, tab, j + 6, q6, pi, si, sx, sy, sz, c2row, drow, v);
        pair_one<DIM, NS, SHIFT>(p, tab, j + 7, q7, pi, si, sx, sy, sz, c2row, drow, v);
    }
    for (; j + 4 <= e; j += 4, qp += 4) {
        const float4 q0 = qp[0], q1 = qp[1], q2 = qp[2], q3 = qp[3];
        pair_one<DIM, NS, SHIFT>(p, tab, j, q0, pi, si, sx, sy, sz, c2row, drow, v);
        pair_one<DIM, NS, SHIFT>(p, tab, j + 1, q1, pi, si, sx, sy, sz, c2row, drow, v);
        pair_one<DIM, NS, SHIFT>(p, tab, j + 2, q2, pi, si, sx, sy, sz, c2row, drow, v);
        pair_one<DIM, NS, SHIFT>(p, tab, j + 3, q3, pi, si, sx, sy, sz, c2row, drow, v);
    }
    for (; j < e; ++j) {
        const float4 q = Ps[j];
        pair_one<DIM, NS, SHIFT>(p, tab, j, q, pi, si, sx, sy, sz, c2row, drow, v);
    }
}

// Repulsion F_i = -sum k (d_ij - r) dx / r over neighbours with r > 0,
// evaluated as k d / r - k with the hardware reciprocal square root, for
// every candidate, and selected without a branch (in dense regions nearly
// every wave has a neighbour among its candidates).  The self pair and
// coincident agents (r2 = 0, dx = 0) contribute exactly zero through the
// product with dx: the clamp below keeps the factor finite there.
struct ForceVisitor {
    float k, fcap;
    float F[3];
    // The factor k (d / r - 1) is positive exactly for overlapping pairs
    // (r < d, up to the rounding of rsq; at r = d the force vanishes), so
    // clamping it to [0, fcap] selects them without a compare.  At r = 0
    // rsq gives +inf and the clamp leaves fcap * dx = 0.
    __device__ __forceinline__ void operator()(uint32_t, float dx, float dy, float dz, float r2,
                                               float, float dd, int) {
        const float fr = fmaf(k * dd, __builtin_amdgcn_rsqf(r2), -k);
        const float f = __builtin_amdgcn_fmed3f(fr, 0.0f, fcap);
        F[0] = fmaf(-f, dx, F[0]);
        F[1] = fmaf(-f, dy, F[1]);
        F[2] = fmaf(-f, dz, F[2]);
    }
};

// Exponential potential u = k exp(-r/d) cut at the pair's range (c2):
// F_i = -sum (k/d) exp(-r/d) dx / r over neighbours with r > 0.
struct ExpVisitor {
    float k;
    float F[3];
    __device__ __forceinline__ void operator()(uint32_t, float dx, float dy, float dz, float r2,
                                               float c2, float dd, int) {
        if (r2 < c2 && r2 > 0.0f) {
            // k / d and log2(e) / d are loop-invariant for one species
            // (hoisted); r / d <= the cut range, so the hardware exp2 and rsq
            // (1 ulp) stay in their normal range
            const float kd = k / dd, l2d = 1.44269504088896341f / dd;
            const float rinv = __builtin_amdgcn_rsqf(r2);
            const float f = kd * __builtin_amdgcn_exp2f(-(r2 * rinv) * l2d) * rinv;
            F[0] = fmaf(-f, dx, F[0]);
            F[1] = fmaf(-f, dy, F[1]);
            F[2] = fmaf(-f, dz, F[2]);
        }
    }
};

// Hard-sphere overlap correction: every pair closer than its contact
// distance d pushes i away from j by 2 (d - r) D_i / (D_i + D_j) (share row
// of species i: share[sj] = 2 D_i / (D_i + D_j), 0 for two immobile agents).
struct OverlapVisitor {
    const float *share;
    float C[3];
    __device__ __forceinline__ void operator()(uint32_t, float dx, float dy, float dz, float r2,
                                               float c2, float dd, int sj) {
        if (r2 < c2 && r2 > 0.0f) {
            const float rinv = rsqrtf(r2);
            const float g = share[sj] * (dd * rinv - 1.0f);
            C[0] = fmaf(-g, dx, C[0]);
            C[1] = fmaf(-g, dy, C[1]);
            C[2] = fmaf(-g, dz, C[2]);
        }
    }
};

// Forces plus the neighbour count and id hash (self excluded).
template <class FV>
struct DebugVisitor {
    FV fv;
    uint32_t self;
    const uint32_t *Is;
    uint32_t cnt;
    unsigned long long hs;
    __device__ __forceinline__ void operator()(uint32_t j, float dx, float dy, float dz, float r2,
                                               float c2, float dd, int sj) {
        if (r2 < c2 && j != self) {
            cnt += 1;
            hs += splitmix64((unsigned long long)Is[j]);
        }
        fv(j, dx, dy, dz, r2, c2, dd, sj);
    }
};

// Nine keys in descending order (a 28-comparator network, Batcher's
// odd-even merge sort of 16 inputs restricted to the first 9).
__device__ __forceinline__ void sort9_desc(uint32_t k[9]) {
    constexpr int kNet[28][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3}, {4, 6},
                                 {5, 7}, {1, 2}, {5, 6}, {0, 4}, {1, 5}, {2, 6}, {3, 7},
                                 {2, 4}, {3, 5}, {1, 2}, {3, 4}, {5, 6}, {0, 8}, {4, 8},
                                 {2, 4}, {3, 5}, {6, 8}, {1, 2}, {3, 4}, {5, 6}, {7, 8}};
#pragma unroll
    for (int c = 0; c < 28; ++c) {
        const uint32_t a = k[kNet[c][0]], b = k[kNet[c][1]];
        k[kNet[c][0]] = max(a, b);
        k[kNet[c][1]] = min(a, b);
    }
}

// Pair loop over the neighbour bins of an agent at position pi.
// dx = x_j - x_i, plus -L / +L for bins reached through the periodic seam:
// for every pair closer than the cutoff this is exactly the minimum image,
// because the seam is crossed iff |x_j - x_i| > L/2 for such pairs.
// Along x, neighbouring bins are adjacent in memory, so each (y, z) row of
// the stencil is one contiguous agent range (two at the seam).
// widest run of x bins a wave may span on the wave-uniform pair path
constexpr int kSpan = 5;

// rowa: this lane's slot of an LDS table of 9 words per lane (stride
// blockDim.x) for the longest-row-first walk; nullptr walks rows in order.
template <int DIM, int NS, int STENCIL, class V>
__device__ __forceinline__ void pair_loop(const StepParams &p, const SpTab &tab,
                                          const float4 *__restrict__ Ps,
                                          const uint32_t *__restrict__ start, uint32_t bin_base,
                                          float4 pi, int si, V &v,
                                          uint32_t *__restrict__ rowa = nullptr) {
    const int nb = p.nb;
    const float pc[3] = {pi.x, pi.y, pi.z};
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    // squared distance from x_i to the lower / upper face of its own bin
    float glo2[3] = {0.f, 0.f, 0.f}, ghi2[3] = {0.f, 0.f, 0.f};
    const float side = p.bin_w;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const float s = fmaxf(pc[a] * p.inv_bin, 0.0f);
        const int b = min((int)s, nb - 1);
        if (STENCIL == 3) {
            lo[a] = b - 1;
            hi[a] = b + 1;
            const float f = fminf(fmaxf(s - (float)b, 0.0f), 1.0f);
            glo2[a] = (f * side) * (f * side);
            ghi2[a] = ((1.0f - f) * side) * ((1.0f - f) * side);
        } else {
            const int up = (s - (float)b) >= 0.5f ? 1 : 0;
            lo[a] = b - 1 + up;
            hi[a] = lo[a] + 1;
        }
    }
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
    // Bins whose nearest face is farther than the largest contact distance
    // of species si cannot hold a neighbour (3^dim stencil only).  The
    // threshold carries a 1e-3 margin over float32 rounding of the faces.
    float cmax2;
    if (NS == 1) {
        cmax2 = c2row[0];
    } else if (NS == 2) {
        cmax2 = fmaxf(c2row[0], c2row[1]);
    } else {
        cmax2 = 0.0f;
        for (int t = 0; t < p.n_species; ++t) cmax2 = fmaxf(cmax2, tab.cut2[si * p.n_species + t]);
    }
    cmax2 *= 1.001f;
    const float L = p.L;
    // When every lane of the wave sits in one (y, z) row of bins and within
    // kSpan adjacent bins along x (the rule in dense clusters, where a bin
    // holds about a wave of agents), every stencil row is one x range common
    // to all lanes: the loop runs on wave-uniform indices (scalar registers).
    // The range covers the lanes' own x bins plus the bin on either side if
    // a lane there can reach it; a lane meets candidates of a bin outside its
    // own stencil only beyond the cutoff, and with nb >= kSpan + 2 the range
    // never holds a bin twice.  A row is skipped only if no lane can reach
    // it.  The span is found with one ballot per offset (active lanes only).
    const int xo = lo[0] + 1;
    const int xf = __builtin_amdgcn_readfirstlane(xo);
    const int yf = __builtin_amdgcn_readfirstlane(lo[1]);
    const int zf = DIM == 3 ? __builtin_amdgcn_readfirstlane(lo[2]) : 0;
    int xmin = xf, xmax = xf;
#pragma unroll
    for (int o = 1; o < kSpan; ++o) {
        if (__any(xo == xf - o)) xmin = xf - o;
        if (__any(xo == xf + o)) xmax = xf + o;
    }
    const bool uniform = STENCIL == 3 && nb >= kSpan + 2 && xmax - xmin < kSpan &&
                         __all(lo[1] == yf && (DIM == 2 || lo[2] == zf) && xo >= xmin &&
                               xo <= xmax);
    if (uniform) {
        const int zlo = zf;
        const int zhi = DIM == 3 ? zlo + 2 : 0;
        const int ylo = yf;
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
            for (int oy = ylo; oy <= ylo + 2; ++oy) {
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
                float d2 = oy < ylo + 1 ? glo2[1] : (oy > ylo + 1 ? ghi2[1] : 0.0f);
                if (DIM == 3) d2 += oz < zlo + 1 ? glo2[2] : (oz > zlo + 1 ? ghi2[2] : 0.0f);
                if (!__any(d2 < cmax2)) continue;
                const int xlo = __any(xo == xmin && d2 + glo2[0] < cmax2) ? xmin - 1 : xmin;
                const int xhi = __any(xo == xmax && d2 + ghi2[0] < cmax2) ? xmax + 1 : xmax;
                const uint32_t row = bin_base + (uint32_t)((qz * nb + qy) * nb);
                const int m0 = max(xlo, 0), m1 = min(xhi, nb - 1);
                const uint32_t a0 = __builtin_amdgcn_readfirstlane(start[row + m0]);
                const uint32_t e0 = __builtin_amdgcn_readfirstlane(start[row + m1 + 1]);
                if (sy == 0.0f && sz == 0.0f)
                    pair_range<DIM, NS, false>(p, tab, Ps, a0, e0, pi, si, 0.f, 0.f, 0.f, c2row,
                                               drow, v);
                else
                    pair_range<DIM, NS, true>(p, tab, Ps, a0, e0, pi, si, 0.f, sy, sz, c2row,
                                              drow, v);
                if (p.periodic) {
                    if (xlo < 0)
                        pair_range<DIM, NS, true>(
                            p, tab, Ps, __builtin_amdgcn_readfirstlane(start[row + xlo + nb]),
                            __builtin_amdgcn_readfirstlane(start[row + nb]), pi, si, -L, sy, sz,
                            c2row, drow, v);
                    if (xhi > nb - 1)
                        pair_range<DIM, NS, true>(
                            p, tab, Ps, __builtin_amdgcn_readfirstlane(start[row]),
                            __builtin_amdgcn_readfirstlane(start[row + xhi - nb + 1]), pi, si, L,
                            sy, sz, c2row, drow, v);
                }
            }
        }
        return;
    }
    // Lanes of one wave walk their own rows in step: each row costs the wave
    // its longest lane.  Outside the periodic seams a lane may walk its rows
    // (9 in 3D, 3 in 2D) longest first instead, which lines up long rows
    // with long rows across the wave (modelled on the initial 1M-agent 3D
    // blob state: 84 instead of 110 candidate slots per wave).  Each row is
    // one x range there.  The order changes only the float summation order
    // of the lane's sum, so it is used only where the caller allows that.
    if (STENCIL == 3 && rowa != nullptr && p.sort_rows) {
        constexpr int R = DIM == 3 ? 9 : 3;   // rows of the stencil
        bool inner = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) inner = inner && lo[a] >= 0 && hi[a] <= nb - 1;
        if (!p.periodic || __all(inner)) {
            // key: length << 5 | row, 16 bits (rows of up to 2047 agents; the
            // row index makes keys distinct); the row's first agent goes to
            // the LDS table.  Every row writes its slot, an empty one 0: the
            // walk reads the slot of empty rows too, and LDS holds whatever
            // the CU's previous work-group left there (a stale first agent
            // near 2^32 would wrap the walk's bound a0 + 8 <= a0 + len).
            const uint32_t bd = blockDim.x;
            uint32_t key[R];
            bool big = false;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int oy = lo[1] + r % 3, oz = DIM == 3 ? lo[2] + r / 3 : 0;
                uint32_t a0 = 0u, len = 0u;
                float d2 = r % 3 == 0 ? glo2[1] : (r % 3 == 2 ? ghi2[1] : 0.0f);
                if (DIM == 3) d2 += r / 3 == 0 ? glo2[2] : (r / 3 == 2 ? ghi2[2] : 0.0f);
                // (a row beyond a wall holds nothing)
                if (oy >= 0 && oy < nb && oz >= 0 && oz < nb && d2 < cmax2) {
                    int xlo = lo[0], xhi = hi[0];
                    if (d2 + glo2[0] >= cmax2) xlo += 1;
                    if (d2 + ghi2[0] >= cmax2) xhi -= 1;
                    const int m0 = max(xlo, 0), m1 = min(xhi, nb - 1);
                    const uint32_t row = bin_base + (uint32_t)((oz * nb + oy) * nb);
                    a0 = start[row + m0];
                    len = start[row + m1 + 1] - a0;
                    big = big || len > 2047u;
                }
                rowa[r * bd] = a0;
                key[r] = (len << 5) | (uint32_t)r;
            }
            if (!__any(big)) {
                if (DIM == 3) {
                    sort9_desc(key);
                } else {
                    // three keys: a three-comparator network
                    uint32_t t = max(key[0], key[1]);
                    key[1] = min(key[0], key[1]);
                    key[0] = t;
                    t = max(key[1], key[R - 1]);
                    key[R - 1] = min(key[1], key[R - 1]);
                    key[1] = t;
                    t = max(key[0], key[1]);
                    key[1] = min(key[0], key[1]);
                    key[0] = t;
                }
                // two keys per register while the rows are walked
                constexpr int NP = (R + 1) / 2;
                uint32_t pk[NP];
#pragma unroll
                for (int q = 0; q < R / 2; ++q) pk[q] = key[2 * q] | (key[2 * q + 1] << 16);
                pk[NP - 1] = key[R - 1];
                uint32_t kk = pk[0] & 0xffffu;
                uint32_t a0 = rowa[(kk & 15u) * bd];
#pragma unroll 1
                for (int k = 0; k < R; ++k) {
                    const uint32_t len = kk >> 5;
                    if (!__any(len != 0u)) break;   // the rest are empty for every lane
                    const uint32_t kn =
                        k < R - 1 ? (pk[(k + 1) >> 1] >> (((k + 1) & 1) * 16)) & 0xffffu : 0u;
                    const uint32_t an = rowa[(kn & 15u) * bd];
                    pair_range<DIM, NS, false, V, 4>(p, tab, Ps, a0, a0 + len, pi, si, 0.f,
                                                     0.f, 0.f, c2row, drow, v);
                    kk = kn;
                    a0 = an;
                }
                return;
            }
        }
    }
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
            int xlo = lo[0], xhi = hi[0];
            if (STENCIL == 3) {
                float d2 = oy < lo[1] + 1 ? glo2[1] : (oy > lo[1] + 1 ? ghi2[1] : 0.0f);
                if (DIM == 3) d2 += oz < lo[2] + 1 ? glo2[2] : (oz > lo[2] + 1 ? ghi2[2] : 0.0f);
                if (d2 >= cmax2) continue;
                if (d2 + glo2[0] >= cmax2) xlo += 1;
                if (d2 + ghi2[0] >= cmax2) xhi -= 1;
            }
            const uint32_t row = bin_base + (uint32_t)((qz * nb + qy) * nb);
            const int m0 = max(xlo, 0), m1 = min(xhi, nb - 1);
            const uint32_t a0 = start[row + m0], e0 = start[row + m1 + 1];
            if (sy == 0.0f && sz == 0.0f)
                pair_range<DIM, NS, false>(p, tab, Ps, a0, e0, pi, si, 0.f, 0.f, 0.f, c2row, drow,
                                           v);
            else
                pair_range<DIM, NS, true>(p, tab, Ps, a0, e0, pi, si, 0.f, sy, sz, c2row, drow,
                                          v);
            if (p.periodic) {
                if (xlo < 0)
                    pair_range<DIM, NS, true>(p, tab, Ps, start[row + xlo + nb], start[row + nb],
                                              pi, si, -L, sy, sz, c2row, drow, v);
                if (xhi > nb - 1)
                    pair_range<DIM, NS, true>(p, tab, Ps, start[row], start[row + xhi - nb + 1],
                                              pi, si, L, sy, sz, c2row, drow, v);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Grid geometry.  Periodic: spacing L/n, nodes i*h, upper corner wraps.
// Walls: spacing L/(n-1), nodes on both walls, lower corner <= n-2.
// ---------------------------------------------------------------------------
// The offset t = x / h - i0 is formed with one rounding, fma(x, 1/h, -i0).
// Where the float32 1/h is exact (an integer for L = 1: 128, 511, 51, ...)
// t is the exact offset rounded once, accurate to an ulp of t rather than
// of x / h.  Where x / h rounds up to an integer k from just below it, the
// floor of the rounded quotient is one too high and t comes out a hair
// below 0: the agent then belongs to cell k - 1 with t = 1 - (that hair).
// The final clamp keeps every weight in [0, 1] (a weight below zero would
// turn into a huge fixed-point deposit), also at a wall's last cell.
struct Cell { int i0, i1; float t; };

__device__ __forceinline__ float cell_offset(float x, float inv_h, float top, float &fi) {
    const float s = fmaxf(x * inv_h, 0.0f);
    fi = fminf(floorf(s), top);
    float t = fmaf(x, inv_h, -fi);
    if (t < 0.0f && fi > 0.0f) {
        fi -= 1.0f;
        t += 1.0f;
    }
    return __builtin_amdgcn_fmed3f(t, 0.0f, 1.0f);
}

__device__ __forceinline__ Cell cell_of(const StepParams &p, float x) {
    float fi;
    Cell c;
    c.t = cell_offset(x, p.inv_h, p.cell_top, fi);
    c.i0 = (int)fi;
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

// Multilinear interpolation of the node values c at x.
template <int DIM>
__device__ __forceinline__ float value_interp(const StepParams &p, const float *__restrict__ c,
                                              float4 x) {
    const Cell cx = cell_of(p, x.x), cy = cell_of(p, x.y);
    const int n = p.grid_n;
    const float wx[2] = {1.0f - cx.t, cx.t}, wy[2] = {1.0f - cy.t, cy.t};
    const int X2[2] = {cx.i0, cx.i1}, Y2[2] = {cy.i0 * n, cy.i1 * n};
    float v = 0.f;
    if (DIM == 2) {
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int a = 0; a < 2; ++a) v = fmaf(wx[a] * wy[b], c[Y2[b] + X2[a]], v);
    } else {
        const Cell cz = cell_of(p, x.z);
        const float wz[2] = {1.0f - cz.t, cz.t};
        const int Z2[2] = {cz.i0 * n * n, cz.i1 * n * n};
#pragma unroll
        for (int e = 0; e < 2; ++e)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int a = 0; a < 2; ++a)
                    v = fmaf(wx[a] * wy[b] * wz[e], c[Z2[e] + Y2[b] + X2[a]], v);
    }
    return v;
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

__device__ __forceinline__ float boundary(const StepParams &p, float x, uint32_t &flag) {
    const float L = p.L;
    if (p.periodic) {
        // x - L floor(x / L), which for x in [-L/2, 3L/2) (a step moves an
        // agent far less than L) is the same single add or subtract
        if (x >= -0.5f * L && x < 1.5f * L) {
            if (x < 0.0f) x += L;
            else if (x >= L) x -= L;
        } else {
            x = x - L * floorf(x / L);
        }
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


// Forward-Euler update of node l with the centred Laplacian (periodic wrap
// or mirror ghost nodes) and the source / uptake densities sigma, upsilon
// at the node.  The particle-in-cell densities are the fixed-point deposits
// divided by the node control volume (the wrapper below); the kernel
// density estimate gives densities directly.
template <int DIM>
__device__ __forceinline__ float pde_node_dens(const PdeParams &q, const float *__restrict__ cb,
                                               const int ic[3], float sigma, float ups,
                                               uint32_t &flag) {
    const int n = q.grid_n, nn = n * n;
    auto nbr = [&](int i, int off) {
        const int r = i + off;
        if (q.periodic) return r < 0 ? r + n : (r >= n ? r - n : r);
        return r < 0 ? 1 : (r >= n ? n - 2 : r);
    };
    const int ix = ic[0], iy = ic[1], iz = ic[2];
    const float c0 = cb[iz * nn + iy * n + ix];
    const int rowo = iz * nn + iy * n;
    float lap = (cb[rowo + nbr(ix, 1)] + cb[rowo + nbr(ix, -1)]) +
                (cb[iz * nn + nbr(iy, 1) * n + ix] + cb[iz * nn + nbr(iy, -1) * n + ix]);
    float diag = 4.0f;
    if (DIM == 3) {
        lap += cb[nbr(iz, 1) * nn + iy * n + ix] + cb[nbr(iz, -1) * nn + iy * n + ix];
        diag = 6.0f;
    }
    lap = (lap - diag * c0) * q.inv_h2;
    const float cn = c0 + q.dts * (q.D_c * lap + sigma - ups * c0 - q.gamma * c0);
    if (!isfinite(cn)) flag |= FLAG_NONFINITE;
    if (q.dts * (q.gamma + ups) >= 1.0f) flag |= FLAG_WARN_POSITIVITY;
    return cn;
}

template <int DIM>
__device__ __forceinline__ float pde_node(const PdeParams &q, const float *__restrict__ cb,
                                          const int ic[3], unsigned long long sS,
                                          unsigned long long sU, uint32_t &flag) {
    const int n = q.grid_n;
    float inv_v = 1.0f;
    if (!q.periodic) {
        if (ic[0] == 0 || ic[0] == n - 1) inv_v *= 2.0f;
        if (ic[1] == 0 || ic[1] == n - 1) inv_v *= 2.0f;
        if (DIM == 3 && (ic[2] == 0 || ic[2] == n - 1)) inv_v *= 2.0f;
    }
    const float dens = q.fx_to_density * inv_v;
    const float sigma = (float)sS * dens;
    const float ups = q.has_uptake ? (float)sU * dens : 0.0f;
    return pde_node_dens<DIM>(q, cb, ic, sigma, ups, flag);
}

// Runs of one bin over consecutive active lanes of a wave (agents come in
// cell order, so a collapsed cluster fills whole waves with one bin): the
// run's first lane, its length and this lane's place in it.  Inactive lanes
// are only the tail of the last wave.
struct WaveRun {
    int head, len, pos;
};

__device__ __forceinline__ WaveRun wave_run(uint32_t b) {
    const int lane = (int)__lane_id();
    const unsigned long long act = __ballot(1);
    const uint32_t prev = __shfl_up(b, 1u, 64);
    const unsigned long long heads = __ballot(lane == 0 || prev != b) | ~act;
    const unsigned long long upto = lane == 63 ? ~0ull : (2ull << lane) - 1ull;
    WaveRun r;
    r.head = 63 - __clzll((long long)(heads & upto));
    const unsigned long long after = heads & ~upto;
    r.len = (after ? __ffsll((long long)after) - 1 : 64) - r.head;
    r.pos = lane - r.head;
    return r;
}


// The counting sort's scatter of agent i (all lanes of the wave that hold
// an agent take part): the bin counted by the kernel that wrote x,
// recomputed from x by the same float32 arithmetic (instance tables are
// equal-sized), its slot taken by counting the bin down, a run of lanes
// with one bin through its first lane's atomic.
template <int DIM>
__device__ __forceinline__ void scatter_agent(const StepParams &p, const float4 *__restrict__ P,
                                              const uint32_t *__restrict__ I,
                                              uint32_t *__restrict__ count,
                                              const uint32_t *__restrict__ start,
                                              float4 *__restrict__ Ps, uint32_t *__restrict__ Is,
                                              int i) {
    const float4 x = P[i];
    const uint32_t b = inst_of(x.w) * (uint32_t)p.bins_per_inst + agent_bin<DIM>(p, x);
    const WaveRun run = wave_run(b);
    uint32_t top = 0;
    if (run.pos == 0) top = atomicSub(count + b, (uint32_t)run.len);
    top = __shfl(top, run.head, 64);
    const uint32_t d = start[b] + top - 1u - (uint32_t)run.pos;
    Ps[d] = x;
    Is[d] = I[i];
}

}  // namespace pc
