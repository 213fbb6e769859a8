// Direct decision (paper Sec. I and III): exact scalar products of each
// receiver's frame with the atoms of eq. (3),
//   D_dir(x, v) = sum_q | sum_m sum_s Y_q[m][s] exp(-j 2 pi (f_r s + f_d m)) |^2,
// evaluated as two contractions per receiver:
//   stage 1 (range zoom): G_q[x][m] = sum_s Y_q[m][s] exp(-j 2 pi f_r(x) s),
//     a [locations x Ms] x [Ms x Mc] complex product with the range atoms
//     generated on the fly;
//   stage 2 (Doppler zoom): per location, sum_m G_q[x][m] exp(-j 2 pi f_d(x, v) m)
//     over the velocity slab, |.|^2, sum over receivers, slab write and block max.
// Phases are held in 32-bit fixed point (cycles modulo one), so s * f_r and
// m * f_d wrap exactly.  This file is the FP32 VALU path.
#include "gh_internal.h"

namespace gh {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxPts = 16;

// Stage 1: one workgroup per (group of `lt` locations, receiver).
__global__ __launch_bounds__(kThreads) void direct_stage1_f32(Geom g, GridP gp, int lt, const float2* __restrict__ y,
                                                             float2* __restrict__ gws) {
    extern __shared__ float2 atoms[];   // [lt][Ms]
    __shared__ uint32_t frq[16];
    const int q = blockIdx.y;
    const int loc0 = blockIdx.x * lt;
    const int ms = g.ms, mc = g.mc;
    if (threadIdx.x < lt) {
        const int loc = loc0 + threadIdx.x;
        uint32_t fr = 0;
        if (loc < gp.nloc) {
            const int ix = loc / gp.n[1], iy = loc - ix * gp.n[1];
            double r, wx, wy;
            bistatic(g, q, gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], r, wx, wy);
            fr = cycles_to_fixed(g.fr_per_m * r);
        }
        frq[threadIdx.x] = fr;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < lt * ms; e += kThreads) {
        const int li = e / ms, s = e - li * ms;
        atoms[e] = (loc0 + li < gp.nloc) ? expm_fixed(frq[li] * (uint32_t)s) : make_float2(0.f, 0.f);
    }
    __syncthreads();
    const float2* yq = y + (size_t)q * mc * ms;
    for (int o = threadIdx.x; o < lt * mc; o += kThreads) {
        const int li = o / mc, m = o - li * mc;
        const int loc = loc0 + li;
        if (loc >= gp.nloc) continue;
        const float2* row = yq + (size_t)m * ms;
        const float2* at = atoms + li * ms;
        float re = 0.f, im = 0.f;
        for (int s = 0; s < ms; ++s) {
            const float2 v = row[s], a = at[s];
            re = fmaf(v.x, a.x, fmaf(-v.y, a.y, re));
            im = fmaf(v.x, a.y, fmaf(v.y, a.x, im));
        }
        gws[((size_t)q * gp.nloc + loc) * mc + m] = make_float2(re, im);
    }
}

// Stage 2: one workgroup per location; threads own the velocity slab.
__global__ __launch_bounds__(kThreads) void direct_stage2_f32(Geom g, GridP gp, const float2* __restrict__ gws,
                                                             float* __restrict__ dec, gh_peak* __restrict__ block,
                                                             const int64_t* __restrict__ excl, int nexcl) {
    extern __shared__ float2 grow[];     // [Mc]
    __shared__ uint32_t ph[kMaxRx][3];
    __shared__ int excl_local[kMaxSupport];
    __shared__ int n_excl_local;
    __shared__ float red_v[kThreads / 64];
    __shared__ int red_i[kThreads / 64];
    const int tid = threadIdx.x;
    const int loc = blockIdx.x;
    const int ix = loc / gp.n[1], iy = loc - ix * gp.n[1];
    const int nv = gp.nv, nvy = gp.n[3], mc = g.mc;
    if (tid < g.k) {
        double r, wx, wy;
        bistatic(g, tid, gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], r, wx, wy);
        ph[tid][0] = cycles_to_fixed(g.fd_per_mps * (wx * gp.lo[2] + wy * gp.lo[3]));
        ph[tid][1] = cycles_to_fixed_step(g.fd_per_mps * wx * gp.step[2]);
        ph[tid][2] = cycles_to_fixed_step(g.fd_per_mps * wy * gp.step[3]);
    }
    if (tid == 0) n_excl_local = local_exclusions(excl, nexcl, loc, nv, excl_local);
    float acc[kMaxPts];
#pragma unroll
    for (int j = 0; j < kMaxPts; ++j) acc[j] = 0.f;
    for (int q = 0; q < g.k; ++q) {
        __syncthreads();
        for (int m = tid; m < mc; m += kThreads) grow[m] = gws[((size_t)q * gp.nloc + loc) * mc + m];
        __syncthreads();
        const uint32_t f0 = ph[q][0], fx = ph[q][1], fy = ph[q][2];
#pragma unroll
        for (int j = 0; j < kMaxPts; ++j) {
            const int v = tid + j * kThreads;
            if (v < nv) {
                const int ivx = v / nvy, ivy = v - ivx * nvy;
                const uint32_t fd = f0 + (uint32_t)ivx * fx + (uint32_t)ivy * fy;
                uint32_t p = 0;
                float re = 0.f, im = 0.f;
                for (int m = 0; m < mc; ++m) {
                    const float2 e = expm_fixed(p);
                    const float2 gv = grow[m];
                    re = fmaf(gv.x, e.x, fmaf(-gv.y, e.y, re));
                    im = fmaf(gv.x, e.y, fmaf(gv.y, e.x, im));
                    p += fd;
                }
                acc[j] = fmaf(re, re, fmaf(im, im, acc[j]));
            }
        }
    }
    __syncthreads();
    slab_epilogue<kThreads, kMaxPts>(acc, nv, loc, dec, block, excl_local, n_excl_local, red_v, red_i);
}

}  // namespace

size_t direct_ws_bytes(const Geom& g, const GridP& gp, int /*gemm*/) {
    return (size_t)g.k * gp.nloc * g.mc * sizeof(float2);
}

hipError_t launch_direct(const Geom& g, const GridP& gp, const float2* y, int gemm, void* ws, float* dec,
                         gh_peak* block, const int64_t* excl, int nexcl, hipStream_t st) {
    (void)gemm;
    float2* gws = static_cast<float2*>(ws);
    int lt = 4096 / g.ms;
    if (lt > 16) lt = 16;
    if (lt < 1) lt = 1;
    hipLaunchKernelGGL(direct_stage1_f32, dim3((gp.nloc + lt - 1) / lt, g.k), dim3(kThreads),
                       (size_t)lt * g.ms * sizeof(float2), st, g, gp, lt, y, gws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(direct_stage2_f32, dim3(gp.nloc), dim3(kThreads), (size_t)g.mc * sizeof(float2), st, g, gp,
                       gws, dec, block, excl, nexcl);
    return hipGetLastError();
}

}  // namespace gh
