// Ensemble statistics of a batch in the style of the experiment of Sect. 4
// (Fig. 1): per-species position histograms summed over every instance and
// the instance-mean chemical field.
#include <hip/hip_runtime.h>

#include "pc_device.h"

namespace pc {

// One thread per agent (grid-stride).  Each work-group counts into an LDS
// copy of the histogram when it fits, then adds its non-zero bins to the
// global one, so global atomics are at most one per agent.  The bin of a
// coordinate is floor(x * s) clamped to [0, m - 1], formed in float32.
template <int DIM, bool LDS>
__global__ void __launch_bounds__(256)
k_species_hist(int n_total, int n_species, const float4 *__restrict__ P, int m, float s,
               int H, uint32_t *__restrict__ counts, uint32_t *__restrict__ totals) {
    extern __shared__ uint32_t lh[];  // n_species * H counts, then n_species totals
    const int nb = n_species * H;
    if (LDS) {
        for (int q = threadIdx.x; q < nb + n_species; q += blockDim.x) lh[q] = 0u;
        __syncthreads();
    }
    const float top = (float)(m - 1);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n_total;
         i += gridDim.x * blockDim.x) {
        const float4 x = P[i];
        const int sp = species_of(x.w);
        const int bx = (int)fminf(fmaxf(floorf(x.x * s), 0.0f), top);
        const int by = (int)fminf(fmaxf(floorf(x.y * s), 0.0f), top);
        int idx = bx + m * by;
        if (DIM == 3) idx += m * m * (int)fminf(fmaxf(floorf(x.z * s), 0.0f), top);
        idx += sp * H;
        if (LDS) {
            atomicAdd(&lh[idx], 1u);
            atomicAdd(&lh[nb + sp], 1u);
        } else {
            atomicAdd(counts + idx, 1u);
            atomicAdd(totals + sp, 1u);
        }
    }
    if (LDS) {
        __syncthreads();
        for (int q = threadIdx.x; q < nb; q += blockDim.x) {
            const uint32_t v = lh[q];
            if (v) atomicAdd(counts + q, v);
        }
        for (int q = threadIdx.x; q < n_species; q += blockDim.x) {
            const uint32_t v = lh[nb + q];
            if (v) atomicAdd(totals + q, v);
        }
    }
}

// Mean over instances of the field, node by node, in FP64.  A work-group
// owns 64 consecutive nodes (one per lane, so every load is a coalesced row
// segment); its W waves split the instances (wave w takes k = w, w + W, ...
// in ascending order) and their partial sums are added in wave order, so
// the result does not depend on scheduling.
constexpr int kMeanWaves = 16;

__global__ void __launch_bounds__(64 * kMeanWaves)
k_field_mean(const float *__restrict__ c, int n_inst, int64_t G, float *__restrict__ out) {
    __shared__ double part[kMeanWaves][64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t l = (int64_t)blockIdx.x * 64 + lane;
    double acc = 0.0;
    if (l < G) {
        int k = wv;
        for (; k + 3 * kMeanWaves < n_inst; k += 4 * kMeanWaves) {
            const float a0 = c[(int64_t)k * G + l];
            const float a1 = c[(int64_t)(k + kMeanWaves) * G + l];
            const float a2 = c[(int64_t)(k + 2 * kMeanWaves) * G + l];
            const float a3 = c[(int64_t)(k + 3 * kMeanWaves) * G + l];
            acc += (double)a0;
            acc += (double)a1;
            acc += (double)a2;
            acc += (double)a3;
        }
        for (; k < n_inst; k += kMeanWaves) acc += (double)c[(int64_t)k * G + l];
    }
    part[wv][lane] = acc;
    __syncthreads();
    if (wv == 0 && l < G) {
        double s = 0.0;
        for (int w = 0; w < kMeanWaves; ++w) s += part[w][lane];
        out[l] = (float)(s / n_inst);
    }
}

constexpr int kHistLdsBytes = 64 * 1024;

int launch_species_hist(const StepParams &p, const Buffers &b, int src, int m, float s,
                        uint32_t *counts, uint32_t *totals, hipStream_t st) {
    int64_t H = 1;
    for (int a = 0; a < p.dim; ++a) H *= m;
    const int64_t nb = p.n_species * H;
    launch_zero_u32(counts, nb, st);
    launch_zero_u32(totals, p.n_species, st);
    const size_t lds = 4 * (size_t)(nb + p.n_species);
    const bool use_lds = lds <= (size_t)kHistLdsBytes;
    // enough work-groups to fill the chip, each with many agents so the LDS
    // flush stays small next to the counting
    int64_t blocks = (p.n_total + 255) / 256;
    if (use_lds && blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    const dim3 g((unsigned)blocks), t(256);
    const size_t sh = use_lds ? lds : 0;
    if (p.dim == 2) {
        if (use_lds)
            hipLaunchKernelGGL((k_species_hist<2, true>), g, t, sh, st, p.n_total, p.n_species,
                               b.P[src], m, s, (int)H, counts, totals);
        else
            hipLaunchKernelGGL((k_species_hist<2, false>), g, t, 0, st, p.n_total, p.n_species,
                               b.P[src], m, s, (int)H, counts, totals);
    } else {
        if (use_lds)
            hipLaunchKernelGGL((k_species_hist<3, true>), g, t, sh, st, p.n_total, p.n_species,
                               b.P[src], m, s, (int)H, counts, totals);
        else
            hipLaunchKernelGGL((k_species_hist<3, false>), g, t, 0, st, p.n_total, p.n_species,
                               b.P[src], m, s, (int)H, counts, totals);
    }
    return 0;
}

void launch_field_mean(const float *c, int n_inst, int64_t G, float *out, hipStream_t st) {
    hipLaunchKernelGGL(k_field_mean, dim3((unsigned)((G + 63) / 64)), dim3(64 * kMeanWaves), 0,
                       st, c, n_inst, G, out);
}

}  // namespace pc
