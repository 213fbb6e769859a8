// Grid-hopping sweep, column kernel (paper Sec. IV, eq. (7)): the variant used
// whenever the velocity slab has a power-of-two number of vy points (8..64),
// at most 32 vx points, and the per-location Doppler tables fit in LDS.
//
// Layout: a workgroup owns `lpb` consecutive locations; thread (l, c) owns the
// vy column c of location l and walks its vx rows.  Along a column the Doppler
// coordinate is t_d(ivx) = t0 + ivy*ay + ivx*ax, so after one multiply per
// (thread, receiver) each point costs one 32-bit add.  The coordinate is held
// in fixed point with 2^32 = 512 bins (N_d <= 512: the map index is the top
// bits masked by N_d - 1, exact because N_d divides 512) or 2^32 = N_d bins
// (N_d > 512); the fraction b becomes the float 1 + b by inserting its top 23
// bits into the mantissa of 1.0.
//
// Per receiver the workgroup first builds the Doppler tables of its locations
// (coalesced: each thread a short contiguous run of entries): the range
// interpolation (2 or 4 map rows, read straight from the maps) collapses to a
// profile h[l], and each segment [l, l+1] stores the Doppler interpolant as a
// polynomial in the fraction:
//   bilinear: I = e' + (1 + b) d,        d = h[l+1] - h[l], e' = h[l] - d
//   bicubic : I = c0 + b c1 + b^2 c2 + b^3 c3   (Keys, a = -1/2)
// Then every point reads one table entry (16 or 32 bytes of LDS), evaluates the
// polynomial and accumulates |I|^2 in a register.  The column loop is fully
// unrolled to a compile-time height NVX (points beyond the slab are evaluated
// on valid table entries and discarded), so the LDS reads of a column are in
// flight together.  The volume and the block maxima are written once, after
// the last receiver.
#include <stdlib.h>

#include "gh_internal.h"

namespace gh {
namespace {

constexpr int kThreads = 256;

struct FastGeo {
    int i0;        // first range row (unwrapped)
    float a;       // fractional range coordinate
    uint32_t t0;   // Doppler coordinate at (vx_lo, vy_lo)
    uint32_t ax;   // per vx step
    uint32_t ay;   // per vy step
};

__device__ __forceinline__ float2 row_at(const float2* __restrict__ mq, const Geom& g, int row, float w, int l,
                                         float2 acc) {
    const int r = row & (g.nr - 1);
    const float s = ((row >> g.log2_nr) & 1) ? g.sign_r * w : w;
    const float2 z = mq[(size_t)r * g.nd + l];
    return make_float2(fmaf(s, z.x, acc.x), fmaf(s, z.y, acc.y));
}

template <int INTERP, int MODE, int NVX>
__global__ __launch_bounds__(kThreads) void gh_sweep_columns(Geom g, GridP gp, int lpb, int log2nvy,
                                                            const float2* __restrict__ maps, float* __restrict__ dec,
                                                            gh_peak* __restrict__ block,
                                                            const int64_t* __restrict__ excl, int nexcl) {
    extern __shared__ float4 lds[];
    constexpr int kEntry = INTERP ? 2 : 1;             // float4 per table entry
    constexpr int kRun = INTERP ? 4 : 2;               // table entries per build run
    const int nd = g.nd;
    float4* tables = lds;                              // [lpb][nd][kEntry]
    FastGeo* geo = reinterpret_cast<FastGeo*>(lds + (size_t)lpb * nd * kEntry);   // [lpb][K]

    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int nvy = 1 << log2nvy;
    const int nvx = gp.n[2];
    const int ll = tid >> log2nvy;
    const int ivy = tid & (nvy - 1);
    // consecutive workgroups go to different XCDs; give each XCD a contiguous run of locations
    const int nb = gridDim.x;
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int per = nb >> 3, extra = nb & 7;
    const int wg = (xcd < extra) ? xcd * (per + 1) + slot : extra * (per + 1) + (xcd - extra) * per + slot;
    const int loc = wg * lpb + ll;
    const bool active = loc < gp.nloc;

    for (int e = tid; e < lpb * g.k; e += nthr) {
        const int l2 = e / g.k, q = e - l2 * g.k;
        const int lc = wg * lpb + l2;
        FastGeo fg = {0, 0.f, 0u, 0u, 0u};
        if (lc < gp.nloc) {
            const int ix = lc / gp.n[1], iy = lc - ix * gp.n[1];
            double r, wx, wy;
            bistatic(g, q, gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], r, wx, wy);
            const double tr = g.kr * r;
            const double fl = floor(tr);
            fg.i0 = (int)fl - (INTERP ? 1 : 0);
            fg.a = (float)(tr - fl);
            const double inv = 1.0 / ((MODE == 0) ? 512.0 : (double)nd);
            fg.t0 = cycles_to_fixed(g.kd * (wx * gp.lo[2] + wy * gp.lo[3]) * inv);
            fg.ax = cycles_to_fixed_step(g.kd * wx * gp.step[2] * inv);
            fg.ay = cycles_to_fixed_step(g.kd * wy * gp.step[3] * inv);
        }
        geo[e] = fg;
    }

    float acc[NVX];
#pragma unroll
    for (int j = 0; j < NVX; ++j) acc[j] = 0.f;

    const float sd = g.sign_d;
    const int runs = (lpb * nd) / kRun;

    for (int q = 0; q < g.k; ++q) {
        __syncthreads();
        const float2* mq = maps + (size_t)q * g.nr * nd;
        for (int run = tid; run < runs; run += nthr) {
            const int first = run * kRun;
            const int lt = first / nd;                 // table (location) of this run
            const int l0 = first - lt * nd;
            const FastGeo fg = geo[lt * g.k + q];
            float4* tab = tables + (size_t)lt * nd * kEntry;
            const float a = fg.a;
            if (INTERP == 0) {
                const float w0 = 1.f - a, w1 = a;
                auto prof = [&](int l) {
                    float sgn = 1.f;
                    if (l >= nd) { l -= nd; sgn = sd; }
                    float2 h = make_float2(0.f, 0.f);
                    h = row_at(mq, g, fg.i0, w0, l, h);
                    h = row_at(mq, g, fg.i0 + 1, w1, l, h);
                    return make_float2(sgn * h.x, sgn * h.y);
                };
                float2 h[kRun + 1];
#pragma unroll
                for (int u = 0; u <= kRun; ++u) h[u] = prof(l0 + u);
#pragma unroll
                for (int u = 0; u < kRun; ++u) {
                    const float2 d = make_float2(h[u + 1].x - h[u].x, h[u + 1].y - h[u].y);
                    tab[l0 + u] = make_float4(h[u].x - d.x, h[u].y - d.y, d.x, d.y);
                }
            } else {
                const float a2 = a * a, a3 = a2 * a;
                const float w0 = -0.5f * a3 + a2 - 0.5f * a;
                const float w1 = 1.5f * a3 - 2.5f * a2 + 1.f;
                const float w2 = -1.5f * a3 + 2.f * a2 + 0.5f * a;
                const float w3 = 0.5f * a3 - 0.5f * a2;
                auto prof = [&](int l) {
                    float sgn = 1.f;
                    if (l < 0) { l += nd; sgn = sd; }
                    else if (l >= nd) { l -= nd; sgn = sd; }
                    float2 h = make_float2(0.f, 0.f);
                    h = row_at(mq, g, fg.i0, w0, l, h);
                    h = row_at(mq, g, fg.i0 + 1, w1, l, h);
                    h = row_at(mq, g, fg.i0 + 2, w2, l, h);
                    h = row_at(mq, g, fg.i0 + 3, w3, l, h);
                    return make_float2(sgn * h.x, sgn * h.y);
                };
                float2 h[kRun + 3];
#pragma unroll
                for (int u = 0; u < kRun + 3; ++u) h[u] = prof(l0 - 1 + u);
#pragma unroll
                for (int u = 0; u < kRun; ++u) {
                    const float2 hm = h[u], h0 = h[u + 1], h1 = h[u + 2], h2 = h[u + 3];
                    const float2 c1 = make_float2(0.5f * (h1.x - hm.x), 0.5f * (h1.y - hm.y));
                    const float2 c2 = make_float2(fmaf(-0.5f, h2.x, fmaf(2.f, h1.x, fmaf(-2.5f, h0.x, hm.x))),
                                                  fmaf(-0.5f, h2.y, fmaf(2.f, h1.y, fmaf(-2.5f, h0.y, hm.y))));
                    const float2 c3 = make_float2(fmaf(0.5f, h2.x - hm.x, 1.5f * (h0.x - h1.x)),
                                                  fmaf(0.5f, h2.y - hm.y, 1.5f * (h0.y - h1.y)));
                    tab[2 * (l0 + u)] = make_float4(h0.x, h0.y, c1.x, c1.y);
                    tab[2 * (l0 + u) + 1] = make_float4(c2.x, c2.y, c3.x, c3.y);
                }
            }
        }
        __syncthreads();
        const FastGeo fg = geo[ll * g.k + q];
        uint32_t t = fg.t0 + (uint32_t)ivy * fg.ay;
        const uint32_t ax = fg.ax;
        const float4* tab = tables + (size_t)ll * nd * kEntry;
        const uint32_t bin_lo = (MODE == 0) ? 23u : (uint32_t)(32 - g.log2_nd);
        const uint32_t fsh = (MODE == 0) ? 0u : (uint32_t)(g.log2_nd - 9);
        constexpr int kBatch = INTERP ? 4 : 8;         // LDS reads kept in flight per column
#pragma unroll
        for (int j0 = 0; j0 < NVX; j0 += kBatch) {
            float4 e0[kBatch], e1[kBatch];
            float b1[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const uint32_t bin = __builtin_amdgcn_ubfe(t, bin_lo, (uint32_t)g.log2_nd);
                b1[u] = __uint_as_float(((t << fsh) & 0x007fffffu) | 0x3f800000u);   // 1 + fraction
                e0[u] = tab[bin * kEntry];
                if (INTERP) e1[u] = tab[bin * kEntry + 1];
                t += ax;
            }
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                float re, im;
                if (INTERP == 0) {
                    re = fmaf(b1[u], e0[u].z, e0[u].x);
                    im = fmaf(b1[u], e0[u].w, e0[u].y);
                } else {
                    const float b = b1[u] - 1.f;
                    re = fmaf(b, e1[u].z, e1[u].x);
                    im = fmaf(b, e1[u].w, e1[u].y);
                    re = fmaf(b, re, e0[u].z);
                    im = fmaf(b, im, e0[u].w);
                    re = fmaf(b, re, e0[u].x);
                    im = fmaf(b, im, e0[u].y);
                }
                acc[j0 + u] = fmaf(re, re, fmaf(im, im, acc[j0 + u]));
            }
        }
    }

    // volume, then the per-location maximum (ties to the lowest index)
    if (!active) return;
    const int nv = gp.nv;
    uint64_t skip = 0;
    for (int e = 0; e < nexcl; ++e) {
        const int64_t d = excl[e] - (int64_t)loc * nv;
        if (d >= 0 && d < nv && (int)(d & (nvy - 1)) == ivy) skip |= 1ull << (int)(d >> log2nvy);
    }
    float bv = -INFINITY;
    int bi = 0x7fffffff;
    float* dl = dec ? dec + (size_t)loc * nv + ivy : nullptr;
#pragma unroll
    for (int j = 0; j < NVX; ++j) {
        if (j < nvx) {
            if (dl) dl[j << log2nvy] = acc[j];
            if (!((skip >> j) & 1) && acc[j] > bv) {
                bv = acc[j];
                bi = (j << log2nvy) + ivy;
            }
        }
    }
    for (int off = nvy >> 1; off >= 1; off >>= 1) {
        const float v2 = __shfl_xor(bv, off, 64);
        const int i2 = __shfl_xor(bi, off, 64);
        peak_merge(bv, bi, v2, i2);
    }
    if (ivy == 0) {
        gh_peak p;
        p.value = bv;
        p.reserved = 0;
        p.index = (int64_t)loc * nv + (bi == 0x7fffffff ? 0 : bi);
        block[loc] = p;
    }
}

template <int INTERP, int MODE>
hipError_t launch_cols(int nvx_t, dim3 grid, dim3 threads, size_t lds, hipStream_t st, const Geom& g,
                       const GridP& gp, int lpb, int log2nvy, const float2* maps, float* dec, gh_peak* block,
                       const int64_t* excl, int nexcl) {
    if (nvx_t == 8)
        hipLaunchKernelGGL((gh_sweep_columns<INTERP, MODE, 8>), grid, threads, lds, st, g, gp, lpb, log2nvy, maps, dec,
                           block, excl, nexcl);
    else if (nvx_t == 16)
        hipLaunchKernelGGL((gh_sweep_columns<INTERP, MODE, 16>), grid, threads, lds, st, g, gp, lpb, log2nvy, maps,
                           dec, block, excl, nexcl);
    else
        hipLaunchKernelGGL((gh_sweep_columns<INTERP, MODE, 32>), grid, threads, lds, st, g, gp, lpb, log2nvy, maps,
                           dec, block, excl, nexcl);
    return hipGetLastError();
}

}  // namespace

// Tile choice: as many locations per workgroup as 256 threads allow, with the
// tables of one receiver within the LDS budget and every wave full.  Returns
// false when the shape needs the generic kernel.
bool sweep_columns_plan(const Geom& g, const GridP& gp, int interp, int& lpb, int& log2nvy, size_t& lds) {
    const int nvy = gp.n[3];
    if (nvy < 8 || nvy > 64 || (nvy & (nvy - 1))) return false;
    if (gp.n[2] > 32) return false;
    if (g.nd < 16) return false;
    log2nvy = 0;
    while ((1 << log2nvy) < nvy) ++log2nvy;
    const size_t entry = interp ? 32 : 16;
    static const long budget_env = [] {
        const char* s = getenv("GH_SWEEP_LDS_KB");   // tuning override of the LDS budget
        return s ? atol(s) : 0L;
    }();
    const size_t lds_budget = (budget_env > 0 ? (size_t)budget_env : 48) * 1024;
    const int cap = kThreads / nvy;
    const int fit = (int)(lds_budget / ((size_t)g.nd * entry + (size_t)g.k * sizeof(FastGeo)));
    lpb = cap < fit ? cap : fit;
    const int full_wave = nvy >= 64 ? 1 : 64 / nvy;   // keep every wave full of locations
    if (lpb >= full_wave) lpb -= lpb % full_wave;
    if (lpb < 1) return false;
    lds = (size_t)lpb * g.nd * entry + (size_t)lpb * g.k * sizeof(FastGeo);
    return true;
}

hipError_t launch_gh_sweep_columns(const Geom& g, const GridP& gp, int lpb, int log2nvy, size_t lds,
                                   const float2* maps, int interp, float* dec, gh_peak* block, const int64_t* excl,
                                   int nexcl, hipStream_t st) {
    const int nblocks = (gp.nloc + lpb - 1) / lpb;
    const dim3 grid(nblocks), threads(lpb << log2nvy);
    const int nvx = gp.n[2];
    const int nvx_t = nvx <= 8 ? 8 : (nvx <= 16 ? 16 : 32);
    const bool small = g.nd <= 512;
    if (interp == GH_INTERP_BICUBIC)
        return small ? launch_cols<1, 0>(nvx_t, grid, threads, lds, st, g, gp, lpb, log2nvy, maps, dec, block, excl, nexcl)
                     : launch_cols<1, 1>(nvx_t, grid, threads, lds, st, g, gp, lpb, log2nvy, maps, dec, block, excl, nexcl);
    return small ? launch_cols<0, 0>(nvx_t, grid, threads, lds, st, g, gp, lpb, log2nvy, maps, dec, block, excl, nexcl)
                 : launch_cols<0, 1>(nvx_t, grid, threads, lds, st, g, gp, lpb, log2nvy, maps, dec, block, excl, nexcl);
}

}  // namespace gh
