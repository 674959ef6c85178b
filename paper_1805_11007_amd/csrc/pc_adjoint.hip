// Reverse mode (adjoint) of the chemotaxis step and the density-mismatch
// loss, for gfx950.
//
// One step maps (X^n, c^n) to (X^{n+1}, c^{n+1}) with the noise fixed by the
// Philox keys:
//   y_i     = X_i + dt (F_i(X) + chi_i I(G c^n)(X_i)) + a_i xi_i
//   X'_i    = B(y_i)                        (periodic wrap or reflection)
//   S       = sum_i q_i W(X'_i)             (piecewise-linear deposit)
//   c^{n+1} = n_sub forward-Euler substeps of eq. pde_c with sigma, upsilon = S / (h^d v)
// Given lambda_X = dL/dX^{n+1} and lambda_c = dL/dc^{n+1}, the kernels below
// produce dL/dX^n, dL/dc^n and the derivatives with respect to
// multiplicative scales of chi, k and D (all species), in this order:
//   k_adj_pde    reverse PDE substeps (transposed stencil), densities' adjoint
//   k_adj_agent  deposit + boundary + drift adjoint per agent, lambda_y,
//                scatter of the node-gradient adjoint, parameter sums
//   k_adj_pair   pair-Jacobian term  dt sum_j J(u_ij) (lambda_y,i - lambda_y,j)
//   k_adj_grad   transposed central difference of the node-gradient adjoint
#include "pc_device.h"

namespace pc {

// Corner node indices, multilinear weights W_m = prod_a w_a and their
// derivatives dW_m/dx_b = (+-1/h) prod_{a != b} w_a at position x.
template <int DIM>
struct Corners {
    int node[1 << DIM];
    float W[1 << DIM];
    float dW[1 << DIM][DIM];
};

template <int DIM>
__device__ __forceinline__ void corners_of(const StepParams &p, float4 x, Corners<DIM> &C) {
    Cell cc[3];
    cc[0] = cell_of(p, x.x);
    cc[1] = cell_of(p, x.y);
    if (DIM == 3) cc[2] = cell_of(p, x.z);
    const int n = p.grid_n;
#pragma unroll
    for (int m = 0; m < (1 << DIM); ++m) {
        float w[DIM], dw[DIM];
        int idx = 0, stride = 1;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const int up = (m >> a) & 1;
            w[a] = up ? cc[a].t : 1.0f - cc[a].t;
            dw[a] = up ? p.inv_h : -p.inv_h;
            idx += (up ? cc[a].i1 : cc[a].i0) * stride;
            stride *= n;
        }
        float W = 1.0f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) W *= w[a];
        C.W[m] = W;
        C.node[m] = idx;
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            float d = dw[b];
#pragma unroll
            for (int a = 0; a < DIM; ++a)
                if (a != b) d *= w[a];
            C.dW[m][b] = d;
        }
    }
}

// Central-difference gradient of c at the 2^dim corners of x's cell
// (periodic wrap or mirror ghost nodes), gc[m][a].
template <int DIM>
__device__ __forceinline__ void corner_gradients(const StepParams &p, const float *__restrict__ c,
                                                 float4 x, float gc[1 << DIM][3]) {
    const Cell cx = cell_of(p, x.x), cy = cell_of(p, x.y);
    const int n = p.grid_n, nn = n * n;
    const int X4[4] = {idx_m1(p, cx.i0), cx.i0, cx.i1, idx_p2(p, cx.i0)};
    const int Y4[4] = {idx_m1(p, cy.i0), cy.i0, cy.i1, idx_p2(p, cy.i0)};
    int Z4[4] = {0, 0, 0, 0};
    if (DIM == 3) {
        const Cell cz = cell_of(p, x.z);
        Z4[0] = idx_m1(p, cz.i0);
        Z4[1] = cz.i0;
        Z4[2] = cz.i1;
        Z4[3] = idx_p2(p, cz.i0);
    }
#pragma unroll
    for (int m = 0; m < (1 << DIM); ++m) {
        const int ux = m & 1, uy = (m >> 1) & 1, uz = DIM == 3 ? (m >> 2) & 1 : 0;
        const int zo = DIM == 3 ? Z4[1 + uz] * nn : 0, yo = Y4[1 + uy] * n, xo = X4[1 + ux];
        gc[m][0] = (c[zo + yo + X4[2 + ux]] - c[zo + yo + X4[ux]]) * p.inv_2h;
        gc[m][1] = (c[zo + Y4[2 + uy] * n + xo] - c[zo + Y4[uy] * n + xo]) * p.inv_2h;
        gc[m][2] = 0.0f;
        if (DIM == 3) gc[m][2] = (c[Z4[2 + uz] * nn + yo + xo] - c[Z4[uz] * nn + yo + xo]) * p.inv_2h;
    }
}

// ---------------------------------------------------------------------------
// Reverse of one PDE substep c_new = c + dt' (D_c Lap c + sigma - ups c - gamma c)
//   mu_out = mu + dt' (D_c Lap^T mu - ups mu - gamma mu)
//   d sigma += dt' mu ;  d ups += -dt' c mu
// Lap^T equals Lap on the torus; with mirror ghosts a neighbour j on a wall
// enters with weight 2.  On the last reversed substep the accumulated
// density adjoints are divided by the control volume h^d v (giving dL/dS)
// and the deposits are cleared.
// ---------------------------------------------------------------------------
template <int DIM>
__global__ void __launch_bounds__(256)
k_adj_pde(PdeParams q, const float *__restrict__ mu_in, float *__restrict__ mu_out,
          const float *__restrict__ cprev, unsigned long long *__restrict__ Ssrc,
          unsigned long long *__restrict__ Supt, float *__restrict__ aSrc,
          float *__restrict__ aUpt, int first, int last) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= q.n_nodes_total) return;
    const int n = q.grid_n, nn = n * n;
    const int64_t G = q.nodes_per_inst;
    const int64_t k = l / G;
    const int loc = (int)(l - k * G);
    const int ic[3] = {loc % n, (loc / n) % n, DIM == 3 ? loc / (n * n) : 0};
    const float *mb = mu_in + k * G;
    const int strides[3] = {1, n, nn};
    const float mu = mb[loc];
    float lapT = 0.0f;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const int i = ic[a];
        const int base = loc - i * strides[a];
        if (q.periodic) {
            const int im = i == 0 ? n - 1 : i - 1, ip = i == n - 1 ? 0 : i + 1;
            lapT += mb[base + im * strides[a]] + mb[base + ip * strides[a]] - 2.0f * mu;
        } else {
            float s = -2.0f * mu;
            if (i > 0) s += (i - 1 == 0 ? 2.0f : 1.0f) * mb[base + (i - 1) * strides[a]];
            if (i < n - 1) s += (i + 1 == n - 1 ? 2.0f : 1.0f) * mb[base + (i + 1) * strides[a]];
            lapT += s;
        }
    }
    lapT *= q.inv_h2;
    float inv_v = 1.0f;
    if (!q.periodic)
        for (int a = 0; a < DIM; ++a)
            if (ic[a] == 0 || ic[a] == n - 1) inv_v *= 2.0f;
    const float dens = q.fx_to_density * inv_v;
    const float ups = q.has_uptake ? (float)Supt[l] * dens : 0.0f;
    mu_out[l] = mu + q.dts * (q.D_c * lapT - ups * mu - q.gamma * mu);
    float as = q.dts * mu, au = -q.dts * cprev[l] * mu;
    if (!first) {
        as += aSrc[l];
        au += aUpt[l];
    }
    if (last) {
        const float iv = q.inv_hd * inv_v;
        aSrc[l] = as * iv;
        aUpt[l] = au * iv;
        Ssrc[l] = 0ull;
        if (q.has_uptake) Supt[l] = 0ull;
    } else {
        aSrc[l] = as;
        aUpt[l] = au;
    }
}

// Parameter derivative accumulation: sum over the work-group (256 threads)
// when all its agents belong to one instance, so that each sum takes one
// device atomic per work-group (the three sums are single addresses, where
// atomics queue); else over the wave when its lanes share an instance, else
// per lane.  Every thread of the work-group calls it (idle ones with zeros);
// thread 0 always holds an agent.
__device__ __forceinline__ void add_dtheta(double *__restrict__ dth, uint32_t inst, bool valid,
                                           double v0, double v1, double v2) {
    __shared__ double part[4][3];
    __shared__ uint32_t inst0;
    if (threadIdx.x == 0) inst0 = inst;
    __syncthreads();
    const uint32_t bfirst = inst0;
    if (__syncthreads_and(!valid || inst == bfirst)) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            v0 += __shfl_xor(v0, d, 64);
            v1 += __shfl_xor(v1, d, 64);
            v2 += __shfl_xor(v2, d, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            part[threadIdx.x >> 6][0] = v0;
            part[threadIdx.x >> 6][1] = v1;
            part[threadIdx.x >> 6][2] = v2;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            double s0 = 0.0, s1 = 0.0, s2 = 0.0;
            for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
                s0 += part[w][0];
                s1 += part[w][1];
                s2 += part[w][2];
            }
            unsafeAtomicAdd(dth + 3 * bfirst + 0, s0);
            unsafeAtomicAdd(dth + 3 * bfirst + 1, s1);
            unsafeAtomicAdd(dth + 3 * bfirst + 2, s2);
        }
        return;
    }
    const uint32_t first = __shfl(inst, 0, 64);
    const bool uniform = __all(!valid || inst == first);
    if (uniform) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            v0 += __shfl_xor(v0, d, 64);
            v1 += __shfl_xor(v1, d, 64);
            v2 += __shfl_xor(v2, d, 64);
        }
        if ((threadIdx.x & 63) == 0) {
            unsafeAtomicAdd(dth + 3 * first + 0, v0);
            unsafeAtomicAdd(dth + 3 * first + 1, v1);
            unsafeAtomicAdd(dth + 3 * first + 2, v2);
        }
    } else if (valid) {
        unsafeAtomicAdd(dth + 3 * inst + 0, v0);
        unsafeAtomicAdd(dth + 3 * inst + 1, v1);
        unsafeAtomicAdd(dth + 3 * inst + 2, v2);
    }
}


template <int DIM, int NS, int STENCIL>
__global__ void __launch_bounds__(256)
k_adj_agent(StepParams p, AdjArgs A, const InstInfo *__restrict__ inst,
            const float4 *__restrict__ Ps, const uint32_t *__restrict__ Is,
            const uint32_t *__restrict__ start, const float *__restrict__ c) {
    __shared__ SpTab tab;
    if (NS == 0) {
        load_tab(p, tab);
        __syncthreads();
    }
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = i < p.n_total;
    double d0 = 0.0, d1 = 0.0, d2 = 0.0;
    uint32_t k = 0;
    if (valid) {
        const float4 pi = Ps[i];
        const uint32_t id = Is[i];
        const int si = species_of(pi.w);
        k = inst_of(pi.w);
        const InstInfo ii = inst[k];
        const size_t row = ii.agent_base + id;
        // recompute the forward update up to the boundary map
        ForceVisitor fv{p.k, p.fcap, {0.f, 0.f, 0.f}};
        if (p.k != 0.0f) pair_loop<DIM, NS, STENCIL>(p, tab, Ps, start, ii.bin_base, pi, si, fv);
        const float chi = sel<NS>(p.chi, tab.chi, si) * ii.chi_scale;
        float Ig[3] = {0.f, 0.f, 0.f}, dI[3][3] = {{0.f}};
        Corners<DIM> C0;
        if (chi != 0.0f) {
            float gc[1 << DIM][3];
            corner_gradients<DIM>(p, c + ii.node_base, pi, gc);
            corners_of<DIM>(p, pi, C0);
#pragma unroll
            for (int m = 0; m < (1 << DIM); ++m)
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    Ig[a] = fmaf(C0.W[m], gc[m][a], Ig[a]);
#pragma unroll
                    for (int b = 0; b < DIM; ++b) dI[a][b] = fmaf(C0.dW[m][b], gc[m][a], dI[a][b]);
                }
        }
        const U4 w = philox4x32_10(A.step, id, ii.stream, 0u, ii.key0, ii.key1);
        float xi[3];
        normals<DIM>(w, xi);
        const float amp = sel<NS>(p.amp, tab.amp, si);
        const float pc[3] = {pi.x, pi.y, pi.z};
        // deposit adjoint at the new position
        float4 xn;
        xn.x = A.xnext[row * DIM + 0];
        xn.y = A.xnext[row * DIM + 1];
        xn.z = DIM == 3 ? A.xnext[row * DIM + 2] : 0.0f;
        xn.w = pi.w;
        const float qs = sel<NS>(p.src_fx, tab.src, si) * 2.3283064365386963e-10f;
        const float qu = p.has_uptake ? sel<NS>(p.upt_fx, tab.upt, si) * 2.3283064365386963e-10f
                                      : 0.0f;
        float lam[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < DIM; ++a) lam[a] = A.lamX_in[row * DIM + a];
        if (qs != 0.0f || qu != 0.0f) {
            Corners<DIM> C1;
            corners_of<DIM>(p, xn, C1);
            const float *as = A.aSrc + ii.node_base, *au = A.aUpt + ii.node_base;
#pragma unroll
            for (int m = 0; m < (1 << DIM); ++m) {
                float g = qs * as[C1.node[m]];
                if (p.has_uptake) g = fmaf(qu, au[C1.node[m]], g);
#pragma unroll
                for (int b = 0; b < DIM; ++b) lam[b] = fmaf(g, C1.dW[m][b], lam[b]);
            }
        }
        // boundary: a reflected component flips the sign of its adjoint
        float ly[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const float y = pc[a] + (p.dt * (fv.F[a] + chi * Ig[a]) + amp * xi[a]);
            const bool refl = !p.periodic && (y < 0.0f || y > p.L);
            ly[a] = refl ? -lam[a] : lam[a];
        }
        // stored in the cell-sorted order, where the pair walk reads it
        A.lamY[i] = make_float4(ly[0], ly[1], ly[2], 0.0f);
        // identity and drift terms of dL/dX^n
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            float v = ly[b];
            if (chi != 0.0f) {
                float s = 0.0f;
#pragma unroll
                for (int a = 0; a < DIM; ++a) s = fmaf(ly[a], dI[a][b], s);
                v = fmaf(p.dt * chi, s, v);
            }
            A.lamX_out[row * DIM + b] = v;
        }
        // node-gradient adjoint (scatter)
        if (chi != 0.0f) {
            float *lg = A.lamG + ii.node_base;
#pragma unroll
            for (int m = 0; m < (1 << DIM); ++m) {
                const float s = p.dt * chi * C0.W[m];
#pragma unroll
                for (int a = 0; a < DIM; ++a)
                    unsafeAtomicAdd(lg + (int64_t)a * A.nodes_total + C0.node[m], s * ly[a]);
            }
        }
        // parameter derivatives (scales of chi, k, D at 1)
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            d0 += (double)(p.dt * chi * Ig[a]) * ly[a];
            d1 += (double)(p.dt * fv.F[a]) * ly[a];
            d2 += (double)(0.5f * amp * xi[a]) * ly[a];
        }
    }
    add_dtheta(A.dth, k, valid, d0, d1, d2);
}

// Pair-Jacobian action J(u) v = k [ (d - r)/r v - (d/r) u_hat (u_hat . v) ]
// summed over neighbours with v = lambda_y,i - lambda_y,j.
struct AdjPairVisitor {
    float k;
    float li[3];
    float acc[3];
    const float4 *lamY;  // cell-sorted, indexed like the candidates
    __device__ __forceinline__ void operator()(uint32_t j, float dx, float dy, float dz, float r2,
                                               float c2, float dd, int) {
        if (r2 < c2 && r2 > 0.0f) {
            const float4 lj = lamY[j];
            const float v0 = li[0] - lj.x;
            const float v1 = li[1] - lj.y;
            const float v2 = li[2] - lj.z;
            const float rinv = rsqrtf(r2);
            const float r = r2 * rinv;
            const float ux = dx * rinv, uy = dy * rinv, uz = dz * rinv;
            const float uv = ux * v0 + uy * v1 + uz * v2;
            const float a = k * (dd - r) * rinv, b = k * dd * rinv * uv;
            acc[0] += a * v0 - b * ux;
            acc[1] += a * v1 - b * uy;
            acc[2] += a * v2 - b * uz;
        }
    }
};

template <int DIM, int NS, int STENCIL>
__global__ void __launch_bounds__(256)
k_adj_pair(StepParams p, const InstInfo *__restrict__ inst, const float4 *__restrict__ Ps,
           const uint32_t *__restrict__ Is, const uint32_t *__restrict__ start,
           const float4 *__restrict__ lamY, float *__restrict__ lamX_out) {
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
    AdjPairVisitor v;
    v.k = p.k;
    v.lamY = lamY;
    const float4 l4 = lamY[i];
    v.li[0] = l4.x;
    v.li[1] = l4.y;
    v.li[2] = l4.z;
    v.acc[0] = v.acc[1] = v.acc[2] = 0.0f;
    pair_loop<DIM, NS, STENCIL>(p, tab, Ps, start, ii.bin_base, pi, si, v);
#pragma unroll
    for (int a = 0; a < DIM; ++a) lamX_out[row * DIM + a] += p.dt * v.acc[a];
}

// dL/dc^n = mu^(0) + G^T lambda_g, G the centred difference: on the torus
// (G^T l)_m = (l_{m-1} - l_{m+1}) / 2h per axis; with mirror ghosts the
// wall rows of G vanish, so only interior neighbours contribute.
template <int DIM>
__global__ void __launch_bounds__(256)
k_adj_grad(PdeParams q, float inv_2h, const float *__restrict__ mu0,
           const float *__restrict__ lamG, float *__restrict__ lamC_out) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= q.n_nodes_total) return;
    const int n = q.grid_n, nn = n * n;
    const int64_t G = q.nodes_per_inst;
    const int64_t k = l / G;
    const int loc = (int)(l - k * G);
    const int ic[3] = {loc % n, (loc / n) % n, DIM == 3 ? loc / (n * n) : 0};
    const int strides[3] = {1, n, nn};
    float s = 0.0f;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const float *lg = lamG + (int64_t)a * q.n_nodes_total + k * G;
        const int i = ic[a];
        const int base = loc - i * strides[a];
        if (q.periodic) {
            const int im = i == 0 ? n - 1 : i - 1, ip = i == n - 1 ? 0 : i + 1;
            s += lg[base + im * strides[a]] - lg[base + ip * strides[a]];
        } else {
            if (i - 1 >= 1 && i - 1 <= n - 2) s += lg[base + (i - 1) * strides[a]];
            if (i + 1 >= 1 && i + 1 <= n - 2) s -= lg[base + (i + 1) * strides[a]];
        }
    }
    lamC_out[l] = mu0[l] + s * inv_2h;
}

// ---------------------------------------------------------------------------
// Density-mismatch loss on a periodic histogram grid of m nodes per axis
// (spacing L/m): rho = piecewise-linear histogram of the positions divided
// by the instance's agent count, smoothed by a separable periodic Gaussian
// (taps given), L = sum (rho_s - target)^2.  Gradient: r = 2 (rho_s - t),
// smoothed again (symmetric taps), gathered back to the agents.
// ---------------------------------------------------------------------------

template <int DIM>
__device__ __forceinline__ void hist_cell(const LossArgs &a, float x, int &i0, int &i1, float &t) {
    float fi;
    t = cell_offset(x, a.inv_hh, (float)(a.m - 1), fi);   // as cell_of
    i0 = (int)fi;
    i1 = i0 + 1 == a.m ? 0 : i0 + 1;
}

template <int DIM>
__global__ void k_loss_hist(LossArgs a, const InstInfo *__restrict__ inst, int n_total,
                            const float4 *__restrict__ P, unsigned long long *__restrict__ hist) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_total) return;
    const float4 x = P[j];
    const int64_t base = (int64_t)inst_of(x.w) * a.H;
    const float xc[3] = {x.x, x.y, x.z};
    int i0[3], i1[3];
    float t[3];
    for (int d = 0; d < DIM; ++d) hist_cell<DIM>(a, xc[d], i0[d], i1[d], t[d]);
#pragma unroll
    for (int mm = 0; mm < (1 << DIM); ++mm) {
        float w = 4294967296.0f;
        int64_t idx = 0, stride = 1;
        for (int d = 0; d < DIM; ++d) {
            const int up = (mm >> d) & 1;
            w *= up ? t[d] : 1.0f - t[d];
            idx += (up ? i1[d] : i0[d]) * stride;
            stride *= a.m;
        }
        const unsigned long long v = (unsigned long long)__float2ull_rn(w);
        if (v) atomicAdd(hist + base + idx, v);
    }
}

// in: fixed-point histogram (first pass, scaled by 2^-32 / N) or float
__global__ void k_loss_smooth(LossArgs a, int axis, int n_inst, const InstInfo *__restrict__ inst,
                              const unsigned long long *__restrict__ hist,
                              const float *__restrict__ in, float *__restrict__ out) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= a.H * n_inst) return;
    const int64_t k = l / a.H;
    const int64_t loc = l - k * a.H;
    int64_t stride = 1;
    for (int d = 0; d < axis; ++d) stride *= a.m;
    const int i = (int)((loc / stride) % a.m);
    const int64_t base = k * a.H + loc - (int64_t)i * stride;
    const float scale = hist ? 2.3283064365386963e-10f / (float)inst[k].n_agents : 1.0f;
    float s = 0.0f;
    for (int q = 0; q < a.n_taps; ++q) {
        int ii = i + q - a.radius;
        ii = ((ii % a.m) + a.m) % a.m;
        const int64_t src = base + (int64_t)ii * stride;
        const float v = hist ? (float)hist[src] * scale : in[src];
        s = fmaf(a.taps[q], v, s);
    }
    out[l] = s;
}

__global__ void k_loss_resid(LossArgs a, int n_inst, const float *__restrict__ rho,
                             const float *__restrict__ target, float *__restrict__ r2,
                             double *__restrict__ loss) {
    const int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool valid = l < a.H * n_inst;
    double v = 0.0;
    int64_t k = 0;
    if (valid) {
        const float d = rho[l] - target[l];
        r2[l] = 2.0f * d;
        v = (double)d * (double)d;
        k = l / a.H;
    }
    const int64_t first = __shfl(k, 0, 64);
    if (__all(!valid || k == first)) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
        if ((threadIdx.x & 63) == 0) unsafeAtomicAdd(loss + first, v);
    } else if (valid) {
        unsafeAtomicAdd(loss + k, v);
    }
}

template <int DIM>
__global__ void k_loss_grad(LossArgs a, const InstInfo *__restrict__ inst, int n_total,
                            const float4 *__restrict__ P, const uint32_t *__restrict__ I,
                            const float *__restrict__ rs, float *__restrict__ dLdX) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n_total) return;
    const float4 x = P[j];
    const uint32_t k = inst_of(x.w);
    const InstInfo ii = inst[k];
    const float *rb = rs + (int64_t)k * a.H;
    const float xc[3] = {x.x, x.y, x.z};
    int i0[3], i1[3];
    float t[3];
    for (int d = 0; d < DIM; ++d) hist_cell<DIM>(a, xc[d], i0[d], i1[d], t[d]);
    float g[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int mm = 0; mm < (1 << DIM); ++mm) {
        float w[3], dw[3];
        int64_t idx = 0, stride = 1;
        for (int d = 0; d < DIM; ++d) {
            const int up = (mm >> d) & 1;
            w[d] = up ? t[d] : 1.0f - t[d];
            dw[d] = up ? a.inv_hh : -a.inv_hh;
            idx += (up ? i1[d] : i0[d]) * stride;
            stride *= a.m;
        }
        const float r = rb[idx];
        for (int b = 0; b < DIM; ++b) {
            float dd = dw[b];
            for (int d = 0; d < DIM; ++d)
                if (d != b) dd *= w[d];
            g[b] = fmaf(r, dd, g[b]);
        }
    }
    const size_t row = ii.agent_base + I[j];
    const float invN = 1.0f / (float)ii.n_agents;
    for (int b = 0; b < DIM; ++b) dLdX[row * DIM + b] = g[b] * invN;
}

__global__ void k_zero_f32(float *__restrict__ d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = 0.0f;
}

__global__ void k_zero_f64(double *__restrict__ d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = 0.0;
}

__global__ void k_zero_u64(unsigned long long *__restrict__ d, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = 0ull;
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
static inline unsigned gridn(int64_t n, int block) { return (unsigned)((n + block - 1) / block); }

void launch_adj_pde(const PdeParams &q, const float *mu_in, float *mu_out, const float *cprev,
                    const Buffers &b, float *aSrc, float *aUpt, int first, int last,
                    hipStream_t s) {
    const dim3 g(gridn(q.n_nodes_total, 256)), t(256);
    if (q.dim == 2)
        hipLaunchKernelGGL(k_adj_pde<2>, g, t, 0, s, q, mu_in, mu_out, cprev, b.S_src, b.S_upt,
                           aSrc, aUpt, first, last);
    else
        hipLaunchKernelGGL(k_adj_pde<3>, g, t, 0, s, q, mu_in, mu_out, cprev, b.S_src, b.S_upt,
                           aSrc, aUpt, first, last);
}

template <int DIM, int NS, int ST>
static void adj_agent(const StepParams &p, const AdjArgs &A, const Buffers &b, int src,
                      const float *c, hipStream_t s) {
    hipLaunchKernelGGL((k_adj_agent<DIM, NS, ST>), dim3(gridn(p.n_total, 256)), dim3(256), 0, s,
                       p, A, b.inst, b.P[src], b.I[src], b.start, c);
}

template <int DIM, int NS, int ST>
static void adj_pair(const StepParams &p, const Buffers &b, int src, const float4 *lamY,
                     float *lamX_out, hipStream_t s) {
    hipLaunchKernelGGL((k_adj_pair<DIM, NS, ST>), dim3(gridn(p.n_total, 256)), dim3(256), 0, s, p,
                       b.inst, b.P[src], b.I[src], b.start, lamY, lamX_out);
}

#define PC_ADJ_DISPATCH(FN, ...)                                                    \
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

void launch_adj_agent(const StepParams &p, const AdjArgs &A, const Buffers &b, int src,
                      const float *c, hipStream_t s) {
    PC_ADJ_DISPATCH(adj_agent, p, A, b, src, c, s);
}

void launch_adj_pair(const StepParams &p, const Buffers &b, int src, const float4 *lamY,
                     float *lamX_out, hipStream_t s) {
    PC_ADJ_DISPATCH(adj_pair, p, b, src, lamY, lamX_out, s);
}

void launch_adj_grad(const PdeParams &q, float inv_2h, const float *mu0, const float *lamG,
                     float *lamC_out, hipStream_t s) {
    const dim3 g(gridn(q.n_nodes_total, 256)), t(256);
    if (q.dim == 2)
        hipLaunchKernelGGL(k_adj_grad<2>, g, t, 0, s, q, inv_2h, mu0, lamG, lamC_out);
    else
        hipLaunchKernelGGL(k_adj_grad<3>, g, t, 0, s, q, inv_2h, mu0, lamG, lamC_out);
}

void launch_zero_f32(float *d, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_zero_f32, dim3(gridn(n, 256)), dim3(256), 0, s, d, n);
}

void launch_zero_f64(double *d, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_zero_f64, dim3(gridn(n, 256)), dim3(256), 0, s, d, n);
}

void launch_zero_u64(unsigned long long *d, int64_t n, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_zero_u64, dim3(gridn(n, 256)), dim3(256), 0, s, d, n);
}

void launch_loss(const LossArgs &a, const StepParams &p, const Buffers &b, int n_inst,
                 const float *target, unsigned long long *hist, float *buf0, float *buf1,
                 double *loss, float *dLdX, float *rho_out, hipStream_t s) {
    const int64_t HN = a.H * n_inst;
    launch_zero_u64(hist, HN, s);
    launch_zero_f64(loss, n_inst, s);
    if (a.dim == 2)
        hipLaunchKernelGGL(k_loss_hist<2>, dim3(gridn(p.n_total, 256)), dim3(256), 0, s, a,
                           b.inst, p.n_total, b.P[0], hist);
    else
        hipLaunchKernelGGL(k_loss_hist<3>, dim3(gridn(p.n_total, 256)), dim3(256), 0, s, a,
                           b.inst, p.n_total, b.P[0], hist);
    // smoothing: first axis reads the fixed-point histogram
    float *cur = buf0, *oth = buf1;
    hipLaunchKernelGGL(k_loss_smooth, dim3(gridn(HN, 256)), dim3(256), 0, s, a, 0, n_inst, b.inst,
                       hist, (const float *)nullptr, cur);
    for (int ax = 1; ax < a.dim; ++ax) {
        hipLaunchKernelGGL(k_loss_smooth, dim3(gridn(HN, 256)), dim3(256), 0, s, a, ax, n_inst,
                           b.inst, (const unsigned long long *)nullptr, cur, oth);
        float *t = cur; cur = oth; oth = t;
    }
    if (rho_out) {
        (void)hipMemcpyAsync(rho_out, cur, 4 * (size_t)HN, hipMemcpyDeviceToDevice, s);
        return;
    }
    hipLaunchKernelGGL(k_loss_resid, dim3(gridn(HN, 256)), dim3(256), 0, s, a, n_inst, cur, target,
                       oth, loss);
    if (!dLdX) return;
    // gradient: smooth the residual back (symmetric taps), gather to agents
    float *r = oth, *o = cur;
    for (int ax = 0; ax < a.dim; ++ax) {
        hipLaunchKernelGGL(k_loss_smooth, dim3(gridn(HN, 256)), dim3(256), 0, s, a, ax, n_inst,
                           b.inst, (const unsigned long long *)nullptr, r, o);
        float *t = r; r = o; o = t;
    }
    if (a.dim == 2)
        hipLaunchKernelGGL(k_loss_grad<2>, dim3(gridn(p.n_total, 256)), dim3(256), 0, s, a,
                           b.inst, p.n_total, b.P[0], b.I[0], r, dLdX);
    else
        hipLaunchKernelGGL(k_loss_grad<3>, dim3(gridn(p.n_total, 256)), dim3(256), 0, s, a,
                           b.inst, p.n_total, b.P[0], b.I[0], r, dLdX);
}

}  // namespace pc
