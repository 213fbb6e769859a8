// Grid-hopping sweep (paper Sec. IV, eq. (7)): for every grid point (x, v)
// and receiver q, the scalar product with the model atom is replaced by an
// interpolation of map q at the continuous coordinates (t_r, t_d), and the
// decision is D(x, v) = sum_q |I_q(x, v)|^2.
//
// Work decomposition: one workgroup per location x; its threads own the
// location's velocity slab.  Everything that depends on (x, q) only is hoisted
// out of the velocity loop:
//   * geometry (FP64): R_q, w_q, hence t_r, the range taps and weights, and the
//     Doppler coordinate as an affine function of the velocity indices,
//     t_d = t0 + ivx*ax + ivy*ay, held in 32-bit fixed point where 2^32 is one
//     period of N_d bins (the wrap of the periodic map is integer overflow and
//     the coordinate is exact to a few 1e-6 bins);
//   * the range interpolation collapses the 2 (or 4) map rows around t_r into a
//     Doppler profile H[l] (LDS);
//   * per Doppler segment [l, l+1] the Doppler interpolant is a polynomial in
//     the fraction b: e + b d (bilinear) or c0 + b c1 + b^2 c2 + b^3 c3 (Keys
//     a = -1/2), whose coefficients are tabulated in LDS.
// Per (point, receiver) the hot loop is then: integer coordinate, one LDS
// table read, a complex Horner step and |.|^2.
// Taps beyond one period of a centred map pick up the factor (-1)^(M-1).
#include <stdlib.h>
#include <string.h>

#include "gh_internal.h"

namespace gh {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxPts = 16;     // velocity points per thread: Nvx*Nvy <= 4096

struct LocGeo {
    int i0;        // first range row tap index (unwrapped)
    float a;       // fractional range coordinate
    uint32_t t0;   // Doppler coordinate of (vx_lo, vy_lo), fixed point
    uint32_t ax;   // increment per vx grid step
    uint32_t ay;   // increment per vy grid step
};

template <int DT>
__device__ __forceinline__ float2 map_row_value(const char* __restrict__ mq, const Geom& g, int row, int l) {
    // value of (unwrapped) range row `row` at Doppler bin l in [0, N_d), storage scale undone
    int wraps = row >> g.log2_nr;                  // floor division (arithmetic shift)
    int r = row & (g.nr - 1);
    float2 v = map_ld1<DT>(mq, (uint32_t)(((size_t)r * g.nd + l) * map_elem_bytes(DT)));
    const float sc = map_scale(g.ms, g.mc, DT);
    if (wraps & 1) v = cscale(v, g.sign_r * sc);
    else if (DT != GH_MAP_C64) v = cscale(v, sc);
    return v;
}

template <int INTERP, int DT>
__global__ __launch_bounds__(kThreads) void gh_sweep_kernel(Geom g, GridP gp, const char* __restrict__ maps,
                                                           float* __restrict__ dec, gh_peak* __restrict__ block,
                                                           const int64_t* __restrict__ excl, int nexcl) {
    extern __shared__ float4 lds[];
    float4* table = lds;                                                   // N_d * (1 or 2) entries
    float2* prof = reinterpret_cast<float2*>(lds + g.nd * (INTERP ? 2 : 1));  // N_d
    __shared__ LocGeo geo[kMaxRx];
    __shared__ int excl_local[kMaxSupport];
    __shared__ int n_excl_local;
    __shared__ float red_v[kThreads / 64];
    __shared__ int red_i[kThreads / 64];

    const int tid = threadIdx.x;
    const int loc = blockIdx.x;
    const int ix = loc / gp.n[1];
    const int iy = loc - ix * gp.n[1];
    const int nv = gp.nv;
    const int nvy = gp.n[3];

    if (tid < g.k) {
        const double x = gp.lo[0] + ix * gp.step[0];
        const double y = gp.lo[1] + iy * gp.step[1];
        double r, wx, wy;
        bistatic(g, tid, x, y, r, wx, wy);
        const double tr = g.kr * r;
        const double fl = floor(tr);
        LocGeo lg;
        lg.i0 = (int)fl - (INTERP ? 1 : 0);
        lg.a = (float)(tr - fl);
        const double inv_nd = 1.0 / g.nd;
        lg.t0 = cycles_to_fixed(g.kd * (wx * gp.lo[2] + wy * gp.lo[3]) * inv_nd);
        lg.ax = cycles_to_fixed_step(g.kd * wx * gp.step[2] * inv_nd);
        lg.ay = cycles_to_fixed_step(g.kd * wy * gp.step[3] * inv_nd);
        geo[tid] = lg;
    }
    if (tid == 0) n_excl_local = local_exclusions(excl, nexcl, loc, nv, excl_local);
    __syncthreads();

    float acc[kMaxPts];
#pragma unroll
    for (int j = 0; j < kMaxPts; ++j) acc[j] = 0.f;

    const int shift = 32 - g.log2_nd;
    for (int q = 0; q < g.k; ++q) {
        const LocGeo lg = geo[q];
        const char* mq = maps + (size_t)q * g.nr * g.nd * map_elem_bytes(DT);
        // range interpolation: Doppler profile of this location
        const float a = lg.a;
        float wr[4];
        if (INTERP == 0) {
            wr[0] = 1.f - a;
            wr[1] = a;
        } else {
            const float a2 = a * a, a3 = a2 * a;
            wr[0] = -0.5f * a3 + a2 - 0.5f * a;
            wr[1] = 1.5f * a3 - 2.5f * a2 + 1.f;
            wr[2] = -1.5f * a3 + 2.f * a2 + 0.5f * a;
            wr[3] = 0.5f * a3 - 0.5f * a2;
        }
        for (int l = tid; l < g.nd; l += kThreads) {
            float2 h = make_float2(0.f, 0.f);
#pragma unroll
            for (int t = 0; t < (INTERP ? 4 : 2); ++t) {
                const float2 z = map_row_value<DT>(mq, g, lg.i0 + t, l);
                h.x += wr[t] * z.x;
                h.y += wr[t] * z.y;
            }
            prof[l] = h;
        }
        __syncthreads();
        // Doppler interpolation: per-segment polynomial coefficients
        for (int l = tid; l < g.nd; l += kThreads) {
            const float sd = g.sign_d;
            const float2 h0 = prof[l];
            const float2 h1 = (l + 1 < g.nd) ? prof[l + 1] : cscale(prof[0], sd);
            if (INTERP == 0) {
                table[l] = make_float4(h0.x, h0.y, h1.x - h0.x, h1.y - h0.y);
            } else {
                const float2 hm = (l > 0) ? prof[l - 1] : cscale(prof[g.nd - 1], sd);
                const float2 h2 = (l + 2 < g.nd) ? prof[l + 2] : cscale(prof[l + 2 - g.nd], sd);
                const float2 c1 = make_float2(0.5f * (h1.x - hm.x), 0.5f * (h1.y - hm.y));
                const float2 c2 = make_float2(hm.x - 2.5f * h0.x + 2.f * h1.x - 0.5f * h2.x,
                                              hm.y - 2.5f * h0.y + 2.f * h1.y - 0.5f * h2.y);
                const float2 c3 = make_float2(-0.5f * hm.x + 1.5f * h0.x - 1.5f * h1.x + 0.5f * h2.x,
                                              -0.5f * hm.y + 1.5f * h0.y - 1.5f * h1.y + 0.5f * h2.y);
                table[2 * l] = make_float4(h0.x, h0.y, c1.x, c1.y);
                table[2 * l + 1] = make_float4(c2.x, c2.y, c3.x, c3.y);
            }
        }
        __syncthreads();
        // velocity slab
#pragma unroll
        for (int j = 0; j < kMaxPts; ++j) {
            const int v = tid + j * kThreads;
            if (v < nv) {
                const int ivx = v / nvy;
                const int ivy = v - ivx * nvy;
                const uint32_t t = lg.t0 + (uint32_t)ivx * lg.ax + (uint32_t)ivy * lg.ay;
                const uint32_t l = t >> shift;
                const float b = __uint2float_rn(t << g.log2_nd) * 2.3283064365386963e-10f;
                float2 iv;
                if (INTERP == 0) {
                    const float4 e = table[l];
                    iv = make_float2(fmaf(b, e.z, e.x), fmaf(b, e.w, e.y));
                } else {
                    const float4 e0 = table[2 * l];
                    const float4 e1 = table[2 * l + 1];
                    float re = fmaf(b, e1.z, e1.x), im = fmaf(b, e1.w, e1.y);
                    re = fmaf(b, re, e0.z);
                    im = fmaf(b, im, e0.w);
                    iv = make_float2(fmaf(b, re, e0.x), fmaf(b, im, e0.y));
                }
                acc[j] = fmaf(iv.x, iv.x, fmaf(iv.y, iv.y, acc[j]));
            }
        }
        __syncthreads();
    }

    slab_epilogue<kThreads, kMaxPts>(acc, nv, loc, dec, block, excl_local, n_excl_local, red_v, red_i);
}

// Global maximum over per-location peaks (one workgroup).
__global__ __launch_bounds__(1024) void peak_final_kernel(const gh_peak* __restrict__ blk, int n,
                                                         gh_peak* __restrict__ out, int64_t* __restrict__ slot,
                                                         unsigned* __restrict__ clear) {
    __shared__ float red_v[16];
    __shared__ long long red_i[16];
    float bv;
    long long bi;
    reduce_block_peaks(blk, n, bv, bi, red_v, red_i);
    if (threadIdx.x == 0) {
        if (out) {
            gh_peak p;
            p.value = bv;
            p.reserved = 0;
            p.index = bi;
            *out = p;
        }
        if (slot) *slot = bi;
        if (clear) *clear = 0u;
    }
}

// Global maximum over per-location peaks, split over up to kSplitWgs
// workgroups: each reduces a contiguous share, stores its result in part[]
// and takes a ticket from `done`; the workgroup holding the last ticket merges
// the shares (ties to the lowest index, as in peak_final_kernel), writes the
// result and sets `done` back to zero.  `done` must be zero when the launch
// starts.  A few release fences replace the latency of one workgroup reading
// every peak.
constexpr int kSplitWgs = 64;
constexpr int kSplitThreads = 256;

__global__ __launch_bounds__(kSplitThreads) void peak_final_split_kernel(const gh_peak* __restrict__ blk, int n,
                                                                       int share, gh_peak* __restrict__ out,
                                                                       int64_t* __restrict__ slot,
                                                                       unsigned* __restrict__ done,
                                                                       gh_peak* __restrict__ part) {
    __shared__ float red_v[kSplitThreads / 64];
    __shared__ long long red_i[kSplitThreads / 64];
    __shared__ int last;
    const int b0 = blockIdx.x * share;
    const int len = min(share, n - b0);
    float bv;
    long long bi;
    reduce_block_peaks(blk + b0, len, bv, bi, red_v, red_i);
    if (threadIdx.x == 0) {
        gh_peak p;
        p.value = bv;
        p.reserved = 0;
        p.index = bi;
        part[blockIdx.x] = p;
        __threadfence();
        last = atomicAdd(done, 1u) == gridDim.x - 1;
    }
    __syncthreads();
    if (!last || threadIdx.x >= 64) return;
    // every other workgroup stored its share before taking its ticket
    __threadfence();
    const int t = threadIdx.x;
    bv = -INFINITY;
    bi = 0x7fffffffffffffffLL;
    if (t < (int)gridDim.x) {
        const gh_peak p = part[t];
        bv = p.value;
        bi = p.index;
    }
    for (int off = 32; off >= 1; off >>= 1) {
        const float v2 = __shfl_xor(bv, off, 64);
        const long long i2 = __shfl_xor(bi, off, 64);
        if (v2 > bv || (v2 == bv && i2 < bi)) {
            bv = v2;
            bi = i2;
        }
    }
    if (t == 0) {
        if (out) {
            gh_peak p;
            p.value = bv;
            p.reserved = 0;
            p.index = bi;
            *out = p;
        }
        if (slot) *slot = bi;
        *done = 0u;
    }
}

template <int DT>
void launch_generic(const Geom& g, const GridP& gp, const char* maps, int interp, float* dec, gh_peak* block,
                    const int64_t* excl, int nexcl, hipStream_t st) {
    const size_t lds = (size_t)g.nd * (interp ? 32 : 16) + (size_t)g.nd * 8;
    if (interp == GH_INTERP_BICUBIC)
        hipLaunchKernelGGL((gh_sweep_kernel<1, DT>), dim3(gp.nloc), dim3(kThreads), lds, st, g, gp, maps, dec, block,
                           excl, nexcl);
    else
        hipLaunchKernelGGL((gh_sweep_kernel<0, DT>), dim3(gp.nloc), dim3(kThreads), lds, st, g, gp, maps, dec, block,
                           excl, nexcl);
}

}  // namespace

hipError_t launch_gh_sweep(const Geom& g, const GridP& gp, const void* maps, int map_dtype, int interp, float* dec,
                           gh_peak* block, const int64_t* excl, int nexcl, hipStream_t st) {
    // the generic kernel for every shape when the test switch asks for it
    const bool generic_only = knob(GH_KNOB_SWEEP_GENERIC) != 0;
    int lpb = 0, log2nvy = 0;
    size_t lds_cols = 0;
    if (!generic_only && sweep_columns_plan(g, gp, interp, lpb, log2nvy, lds_cols))
        return launch_gh_sweep_columns(g, gp, lpb, log2nvy, lds_cols, maps, map_dtype, interp, dec, block, excl, nexcl,
                                       st);
    const char* m = static_cast<const char*>(maps);
    if (map_dtype == GH_MAP_F16)
        launch_generic<GH_MAP_F16>(g, gp, m, interp, dec, block, excl, nexcl, st);
    else if (map_dtype == GH_MAP_BF16)
        launch_generic<GH_MAP_BF16>(g, gp, m, interp, dec, block, excl, nexcl, st);
    else
        launch_generic<GH_MAP_C64>(g, gp, m, interp, dec, block, excl, nexcl, st);
    return hipGetLastError();
}

hipError_t launch_peak_final(const gh_peak* block, int nblock, gh_peak* out, int64_t* support_slot, hipStream_t st,
                             unsigned* clear) {
    hipLaunchKernelGGL(peak_final_kernel, dim3(1), dim3(1024), 0, st, block, nblock, out, support_slot, clear);
    return hipGetLastError();
}

size_t peak_split_ws_bytes() { return 256 + kSplitWgs * sizeof(gh_peak); }

hipError_t launch_peak_final_split(const gh_peak* block, int nblock, gh_peak* out, int64_t* support_slot, void* ws,
                                   hipStream_t st) {
    // shares of 16 peaks per thread (one load batch), 4 for small inputs, at most kSplitWgs shares
    const int64_t n = nblock;
    int64_t share = 16 * kSplitThreads;
    if ((n + share - 1) / share < kSplitWgs / 4) share = 4 * kSplitThreads;
    if ((n + share - 1) / share > kSplitWgs) share = (n + kSplitWgs - 1) / kSplitWgs;
    const int nwg = (int)((n + share - 1) / share);
    unsigned* done = static_cast<unsigned*>(ws);
    gh_peak* part = reinterpret_cast<gh_peak*>(static_cast<char*>(ws) + 256);
    hipLaunchKernelGGL(peak_final_split_kernel, dim3(nwg), dim3(kSplitThreads), 0, st, block, nblock, (int)share,
                       out, support_slot, done, part);
    return hipGetLastError();
}

}  // namespace gh
