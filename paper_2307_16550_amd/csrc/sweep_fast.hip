// Grid-hopping sweep, column kernel (paper Sec. IV, eq. (7)): the variant used
// whenever the velocity slab has a power-of-two number of vy points (1..64),
// each thread's share of the vx axis is at most 32 points, and the
// per-location Doppler tables fit in LDS.
//
// Layout: a workgroup owns `lpb` consecutive locations, one per wave (so one
// 8 KB table per wave for N_d = 512, which keeps ~20 waves resident per CU).
// Lane (p, c) of a wave owns the vy column c of its location over the p-th
// run of vx rows.  Along a column the Doppler coordinate is
// t_d(ivx) = t0 + ivy*ay + ivx*ax, so after two multiplies per
// (thread, receiver) each point costs one 32-bit add.  The coordinate is held
// in fixed point with 2^32 = 512 bins (N_d <= 512: the map index is the top
// bits masked by N_d - 1, exact because N_d divides 512) or 2^32 = N_d bins
// (N_d > 512); the fraction b becomes the float 1 + b by inserting its top 23
// bits into the mantissa of 1.0.
//
// Per receiver each wave first builds its location's Doppler table in its own
// LDS slice (coalesced: each lane builds runs of 2 (bilinear) or 4 (bicubic)
// entries from vector loads straight from the maps, range rows and their wrap
// signs resolved once per location; the next receiver's map values are
// prefetched into registers while the current table is evaluated): the range
// interpolation (2 or 4 map rows) collapses to a profile h[l], and each
// segment [l, l+1] stores the Doppler interpolant as a polynomial in the
// fraction:
//   bilinear: I = e' + (1 + b) d,        d = h[l+1] - h[l], e' = h[l] - d
//   bicubic : I = c0 + b c1 + b^2 c2 + b^3 c3   (Keys, a = -1/2)
// Then every point reads one table entry (16 or 32 bytes of LDS), evaluates the
// polynomial and accumulates |I|^2 in a register.  The column loop is fully
// unrolled to a compile-time height NVX (points beyond the slab are evaluated
// on valid table entries and discarded) with its LDS reads issued in batches.
// The volume and the block maxima are written once, after the last receiver.
// Maps stored as 16-bit float pairs (Z / (Ms Mc)) are widened to FP32 in the
// table build, with the storage scale folded into the range weights.
#include <stdlib.h>

#include "gh_internal.h"

namespace gh {
namespace {

constexpr int kThreads = 256;

struct FastGeo {
    uint32_t row[4];   // element offset of each range tap row (row index mod N_r, times N_d)
    float w[4];        // range weights with the wrap sign folded in
    uint32_t t0;       // Doppler coordinate at (vx_lo, vy_lo)
    uint32_t ax;       // per vx step
    uint32_t ay;       // per vy step
    uint32_t pad;
};


__device__ __forceinline__ float2 wsum2(float w0, float2 a, float w1, float2 b) {
    return make_float2(fmaf(w1, b.x, w0 * a.x), fmaf(w1, b.y, w0 * a.y));
}

template <int INTERP, int MODE, int NVX, int DT>
__global__ __launch_bounds__(kThreads) void gh_sweep_columns(Geom g, GridP gp, int lpb, int log2nvy,
                                                            const char* __restrict__ maps, float* __restrict__ dec,
                                                            gh_peak* __restrict__ block,
                                                            const int64_t* __restrict__ excl, int nexcl) {
    extern __shared__ float4 lds[];
    constexpr int kEntry = INTERP ? 2 : 1;             // float4 per table entry
    constexpr int kTaps = INTERP ? 4 : 2;
    const int nd = g.nd;
    const int log2nd = g.log2_nd;
    constexpr int kEs = map_elem_bytes(DT);            // bytes per stored map value
    const float scale = map_scale(g.ms, g.mc, DT);     // folded into the range weights
    float4* tables = lds;                              // [lpb][nd][kEntry]
    FastGeo* geo = reinterpret_cast<FastGeo*>(lds + (size_t)lpb * nd * kEntry);   // [lpb][K]

    const int tid = threadIdx.x;
    const int nvy = 1 << log2nvy;
    const int nvx = gp.n[2];
    // one location per wave: lane = (part, ivy); part p of the wave owns vx rows [p*chunk, (p+1)*chunk)
    const int ll = tid >> 6;
    const int lane = tid & 63;
    const int ivy = lane & (nvy - 1);
    const int part = lane >> log2nvy;
    const int chunk = (nvx + (64 >> log2nvy) - 1) >> (6 - log2nvy);
    const int ivx0 = part * chunk;
    // consecutive workgroups go to different XCDs; give each XCD a contiguous run of locations
    const int nb = gridDim.x;
    const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
    const int per = nb >> 3, extra = nb & 7;
    const int wg = (xcd < extra) ? xcd * (per + 1) + slot : extra * (per + 1) + (xcd - extra) * per + slot;
    const int loc = wg * lpb + ll;
    const bool active = loc < gp.nloc;

    // Geometry of the workgroup's (location, receiver) pairs, one pair per thread;
    // after this single barrier each wave owns its location's table.
    for (int e = tid; e < lpb * g.k; e += blockDim.x) {
        const int lc = wg * lpb + e / g.k;
        const int q = e - (e / g.k) * g.k;
        FastGeo fg;
        for (int u = 0; u < 4; ++u) {
            fg.row[u] = 0;
            fg.w[u] = 0.f;
        }
        fg.t0 = fg.ax = fg.ay = fg.pad = 0;
        if (lc < gp.nloc) {
            const int ix = lc / gp.n[1], iy = lc - ix * gp.n[1];
            double r, wx, wy;
            bistatic(g, q, gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], r, wx, wy);
            const double tr = g.kr * r;
            const double fl = floor(tr);
            const float a = (float)(tr - fl);
            const int i0 = (int)fl - (INTERP ? 1 : 0);
            float w[4];
            if (INTERP == 0) {
                w[0] = 1.f - a;
                w[1] = a;
            } else {
                const float a2 = a * a, a3 = a2 * a;
                w[0] = -0.5f * a3 + a2 - 0.5f * a;
                w[1] = 1.5f * a3 - 2.5f * a2 + 1.f;
                w[2] = -1.5f * a3 + 2.f * a2 + 0.5f * a;
                w[3] = 0.5f * a3 - 0.5f * a2;
            }
            for (int u = 0; u < kTaps; ++u) {
                const int row = i0 + u;
                fg.row[u] = ((uint32_t)(row & (g.nr - 1)) << log2nd) * (uint32_t)kEs;   // byte offset of the row
                fg.w[u] = (((row >> g.log2_nr) & 1) ? g.sign_r * w[u] : w[u]) * scale;
            }
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
    constexpr int kRun = INTERP ? 4 : 2;               // table entries per build run (2: lanes read contiguous float4)
    const int runs = nd / kRun;                        // table runs of this wave's location
    __syncthreads();

    // Bilinear builds are software-pipelined: the map rows of receiver q+1 are
    // loaded into registers while the points of receiver q are evaluated.
    constexpr int kPre = 4;                            // runs per lane held in registers
    const int rpl = (runs + 63) >> 6;
    const bool pipelined = (INTERP == 0) && rpl <= kPre;
    float4 pa[kPre], pb[kPre];
    float2 pa2[kPre], pb2[kPre];
    auto prefetch = [&](int qq) {
        const char* mqq = maps + (size_t)qq * g.nr * nd * kEs;
        const FastGeo fq = geo[ll * g.k + qq];
#pragma unroll
        for (int i = 0; i < kPre; ++i) {
            const int run = lane + 64 * i;
            if (i < rpl && run < runs) {
                const int l0 = run * 2;
                const uint32_t o0 = (uint32_t)l0 * kEs;
                const uint32_t ohi = (l0 + 2 == nd) ? 0u : o0 + 2u * kEs;
                pa[i] = map_ld2<DT>(mqq, fq.row[0] + o0);
                pb[i] = map_ld2<DT>(mqq, fq.row[1] + o0);
                pa2[i] = map_ld1<DT>(mqq, fq.row[0] + ohi);
                pb2[i] = map_ld1<DT>(mqq, fq.row[1] + ohi);
            }
        }
    };
    if (pipelined) prefetch(0);

    for (int q = 0; q < g.k; ++q) {
        // all lanes finished reading the previous receiver's table (in-order LDS per wave)
        __builtin_amdgcn_wave_barrier();
        const char* mq = maps + (size_t)q * g.nr * nd * kEs;
        const FastGeo fb = geo[ll * g.k + q];
        float4* tabl = tables + (size_t)ll * nd * kEntry;
        if (pipelined) {
            const float w0 = fb.w[0], w1 = fb.w[1];
#pragma unroll
            for (int i = 0; i < kPre; ++i) {
                const int run = lane + 64 * i;
                if (i < rpl && run < runs) {
                    const int l0 = run * 2;
                    const float shi = (l0 + 2 == nd) ? sd : 1.f;
                    const float2 h0 = wsum2(w0, make_float2(pa[i].x, pa[i].y), w1, make_float2(pb[i].x, pb[i].y));
                    const float2 h1 = wsum2(w0, make_float2(pa[i].z, pa[i].w), w1, make_float2(pb[i].z, pb[i].w));
                    const float2 h2 = wsum2(w0 * shi, pa2[i], w1 * shi, pb2[i]);
                    const float2 d0 = make_float2(h1.x - h0.x, h1.y - h0.y);
                    const float2 d1 = make_float2(h2.x - h1.x, h2.y - h1.y);
                    tabl[l0] = make_float4(h0.x - d0.x, h0.y - d0.y, d0.x, d0.y);
                    tabl[l0 + 1] = make_float4(h1.x - d1.x, h1.y - d1.y, d1.x, d1.y);
                }
            }
        }
        for (int run = pipelined ? runs : lane; run < runs; run += 64) {
            const int l0 = run * kRun;
            float4* tab = tabl + (size_t)l0 * kEntry;
            // profile values h[l0 - 1 .. l0 + 5]; indices past the period come from its start with sign sd
            const bool top = (l0 + kRun == nd);
            const uint32_t ohi = top ? 0u : (uint32_t)(l0 + kRun) * kEs;
            const float shi = top ? sd : 1.f;
            const uint32_t o0 = (uint32_t)l0 * kEs;
            float2 h[kRun + 3];
            if (INTERP == 0) {
                const float w0 = fb.w[0], w1 = fb.w[1];
#pragma unroll
                for (int u = 0; u < kRun / 2; ++u) {
                    const float4 a = map_ld2<DT>(mq, fb.row[0] + o0 + 2u * kEs * u);
                    const float4 b = map_ld2<DT>(mq, fb.row[1] + o0 + 2u * kEs * u);
                    h[2 * u + 1] = wsum2(w0, make_float2(a.x, a.y), w1, make_float2(b.x, b.y));
                    h[2 * u + 2] = wsum2(w0, make_float2(a.z, a.w), w1, make_float2(b.z, b.w));
                }
                const float2 a2 = map_ld1<DT>(mq, fb.row[0] + ohi);
                const float2 b2 = map_ld1<DT>(mq, fb.row[1] + ohi);
                h[kRun + 1] = wsum2(w0 * shi, a2, w1 * shi, b2);
#pragma unroll
                for (int u = 0; u < kRun; ++u) {
                    const float2 d = make_float2(h[u + 2].x - h[u + 1].x, h[u + 2].y - h[u + 1].y);
                    tab[u] = make_float4(h[u + 1].x - d.x, h[u + 1].y - d.y, d.x, d.y);
                }
            } else {
                const bool bottom = (l0 == 0);
                const uint32_t olo = bottom ? (uint32_t)(nd - 1) * kEs : o0 - kEs;
                const float slo = bottom ? sd : 1.f;
#pragma unroll
                for (int u = 0; u < kRun + 3; ++u) h[u] = make_float2(0.f, 0.f);
#pragma unroll
                for (int tap = 0; tap < 4; ++tap) {
                    const uint32_t rb = fb.row[tap];
                    const float w = fb.w[tap];
                    const float2 v0 = map_ld1<DT>(mq, rb + olo);
                    const float4 v1 = map_ld2<DT>(mq, rb + o0);
                    const float4 v2 = map_ld2<DT>(mq, rb + o0 + 2u * kEs);
                    const float4 v3 = map_ld2<DT>(mq, rb + ohi);
                    const float wl = w * slo, wh = w * shi;
                    h[0] = make_float2(fmaf(wl, v0.x, h[0].x), fmaf(wl, v0.y, h[0].y));
                    h[1] = make_float2(fmaf(w, v1.x, h[1].x), fmaf(w, v1.y, h[1].y));
                    h[2] = make_float2(fmaf(w, v1.z, h[2].x), fmaf(w, v1.w, h[2].y));
                    h[3] = make_float2(fmaf(w, v2.x, h[3].x), fmaf(w, v2.y, h[3].y));
                    h[4] = make_float2(fmaf(w, v2.z, h[4].x), fmaf(w, v2.w, h[4].y));
                    h[5] = make_float2(fmaf(wh, v3.x, h[5].x), fmaf(wh, v3.y, h[5].y));
                    h[6] = make_float2(fmaf(wh, v3.z, h[6].x), fmaf(wh, v3.w, h[6].y));
                }
#pragma unroll
                for (int u = 0; u < kRun; ++u) {
                    const float2 hm = h[u], h0 = h[u + 1], h1 = h[u + 2], h2 = h[u + 3];
                    const float2 c1 = make_float2(0.5f * (h1.x - hm.x), 0.5f * (h1.y - hm.y));
                    const float2 c2 = make_float2(fmaf(-0.5f, h2.x, fmaf(2.f, h1.x, fmaf(-2.5f, h0.x, hm.x))),
                                                  fmaf(-0.5f, h2.y, fmaf(2.f, h1.y, fmaf(-2.5f, h0.y, hm.y))));
                    const float2 c3 = make_float2(fmaf(0.5f, h2.x - hm.x, 1.5f * (h0.x - h1.x)),
                                                  fmaf(0.5f, h2.y - hm.y, 1.5f * (h0.y - h1.y)));
                    tab[2 * u] = make_float4(h0.x, h0.y, c1.x, c1.y);
                    tab[2 * u + 1] = make_float4(c2.x, c2.y, c3.x, c3.y);
                }
            }
        }
        // the table is private to the wave: its LDS writes only have to land before the wave reads them
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (pipelined && q + 1 < g.k) prefetch(q + 1);
        const FastGeo fg = geo[ll * g.k + q];
        uint32_t t = fg.t0 + (uint32_t)ivy * fg.ay + (uint32_t)ivx0 * fg.ax;
        const uint32_t ax = fg.ax;
        const float4* tab = tables + (size_t)ll * nd * kEntry;
        const uint32_t bin_lo = (MODE == 0) ? 23u : (uint32_t)(32 - log2nd);
        const uint32_t fsh = (MODE == 0) ? 0u : (uint32_t)(log2nd - 9);
        constexpr int kWant = INTERP ? 4 : 8;          // LDS reads kept in flight per column
        constexpr int kBatch = NVX < kWant ? NVX : kWant;
#pragma unroll
        for (int j0 = 0; j0 < NVX; j0 += kBatch) {
            float4 e0[kBatch], e1[kBatch];
            float b1[kBatch];
#pragma unroll
            for (int u = 0; u < kBatch; ++u) {
                const uint32_t bin = __builtin_amdgcn_ubfe(t, bin_lo, (uint32_t)log2nd);
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
    uint64_t skip = 0;      // bit j: point (ivx0 + j, ivy) is excluded from the maximum
    for (int e = 0; e < nexcl; ++e) {
        const int64_t d = excl[e] - (int64_t)loc * nv;
        if (d >= 0 && d < nv && (int)(d & (nvy - 1)) == ivy) {
            const int j = (int)(d >> log2nvy) - ivx0;
            if (j >= 0 && j < NVX) skip |= 1ull << j;
        }
    }
    const int jmax = (chunk < nvx - ivx0) ? chunk : nvx - ivx0;   // points of this thread inside the slab
    if (dec) {
        float* dl = dec + (size_t)loc * nv + ((size_t)ivx0 << log2nvy) + ivy;
#pragma unroll
        for (int j = 0; j < NVX; ++j)
            if (j < jmax) dl[j << log2nvy] = acc[j];
    }
    if (nexcl > 0) {
#pragma unroll
        for (int j = 0; j < NVX; ++j)
            if ((skip >> j) & 1) acc[j] = -INFINITY;
    }
    float bv = -INFINITY;
    int bj = -1;
#pragma unroll
    for (int j = 0; j < NVX; ++j) {
        if (j < jmax && acc[j] > bv) {
            bv = acc[j];
            bj = j;
        }
    }
    int bi = bj < 0 ? 0x7fffffff : ((ivx0 + bj) << log2nvy) + ivy;
    for (int off = 32; off >= 1; off >>= 1) {
        const float v2 = __shfl_xor(bv, off, 64);
        const int i2 = __shfl_xor(bi, off, 64);
        peak_merge(bv, bi, v2, i2);
    }
    if (lane == 0) {
        gh_peak p;
        p.value = bv;
        p.reserved = 0;
        p.index = (int64_t)loc * nv + (bi == 0x7fffffff ? 0 : bi);
        block[loc] = p;
    }
}

template <int INTERP, int MODE, int DT>
hipError_t launch_cols(int nvx_t, dim3 grid, dim3 threads, size_t lds, hipStream_t st, const Geom& g,
                       const GridP& gp, int lpb, int log2nvy, const char* maps, float* dec, gh_peak* block,
                       const int64_t* excl, int nexcl) {
    if (nvx_t == 2)
        hipLaunchKernelGGL((gh_sweep_columns<INTERP, MODE, 2, DT>), grid, threads, lds, st, g, gp, lpb, log2nvy, maps,
                           dec, block, excl, nexcl);
    else if (nvx_t == 4)
        hipLaunchKernelGGL((gh_sweep_columns<INTERP, MODE, 4, DT>), grid, threads, lds, st, g, gp, lpb, log2nvy, maps,
                           dec, block, excl, nexcl);
    else if (nvx_t == 8)
        hipLaunchKernelGGL((gh_sweep_columns<INTERP, MODE, 8, DT>), grid, threads, lds, st, g, gp, lpb, log2nvy, maps,
                           dec, block, excl, nexcl);
    else if (nvx_t == 16)
        hipLaunchKernelGGL((gh_sweep_columns<INTERP, MODE, 16, DT>), grid, threads, lds, st, g, gp, lpb, log2nvy, maps,
                           dec, block, excl, nexcl);
    else
        hipLaunchKernelGGL((gh_sweep_columns<INTERP, MODE, 32, DT>), grid, threads, lds, st, g, gp, lpb, log2nvy, maps,
                           dec, block, excl, nexcl);
    return hipGetLastError();
}

template <int DT>
hipError_t launch_cols_dt(int interp, bool small, int nvx_t, dim3 grid, dim3 threads, size_t lds, hipStream_t st,
                          const Geom& g, const GridP& gp, int lpb, int log2nvy, const char* maps, float* dec,
                          gh_peak* block, const int64_t* excl, int nexcl) {
    if (interp == GH_INTERP_BICUBIC)
        return small ? launch_cols<1, 0, DT>(nvx_t, grid, threads, lds, st, g, gp, lpb, log2nvy, maps, dec, block, excl, nexcl)
                     : launch_cols<1, 1, DT>(nvx_t, grid, threads, lds, st, g, gp, lpb, log2nvy, maps, dec, block, excl, nexcl);
    return small ? launch_cols<0, 0, DT>(nvx_t, grid, threads, lds, st, g, gp, lpb, log2nvy, maps, dec, block, excl, nexcl)
                 : launch_cols<0, 1, DT>(nvx_t, grid, threads, lds, st, g, gp, lpb, log2nvy, maps, dec, block, excl, nexcl);
}

}  // namespace

// Tile choice: as many locations per workgroup as 256 threads allow, with the
// tables of one receiver within the LDS budget and every wave full.  Returns
// false when the shape needs the generic kernel.
bool sweep_columns_plan(const Geom& g, const GridP& gp, int interp, int& lpb, int& log2nvy, size_t& lds) {
    const int nvy = gp.n[3];
    if (nvy < 1 || nvy > 64 || (nvy & (nvy - 1))) return false;
    log2nvy = 0;
    while ((1 << log2nvy) < nvy) ++log2nvy;
    const int chunk = (gp.n[2] + (64 >> log2nvy) - 1) >> (6 - log2nvy);   // vx rows per thread
    if (chunk > 32) return false;
    if (g.nd < 16) return false;
    const size_t entry = interp ? 32 : 16;
    static const long budget_env = [] {
        const char* s = getenv("GH_SWEEP_LDS_KB");   // tuning override of the LDS budget
        return s ? atol(s) : 0L;
    }();
    const size_t lds_budget = (budget_env > 0 ? (size_t)budget_env : 40) * 1024;
    const int cap = kThreads / 64;                   // one location per wave
    const int fit = (int)(lds_budget / ((size_t)g.nd * entry + (size_t)g.k * sizeof(FastGeo)));
    lpb = cap < fit ? cap : fit;
    if (lpb < 1) return false;
    lds = (size_t)lpb * g.nd * entry + (size_t)lpb * g.k * sizeof(FastGeo);
    return true;
}

hipError_t launch_gh_sweep_columns(const Geom& g, const GridP& gp, int lpb, int log2nvy, size_t lds,
                                   const void* maps_v, int map_dtype, int interp, float* dec, gh_peak* block,
                                   const int64_t* excl, int nexcl, hipStream_t st) {
    const char* maps = static_cast<const char*>(maps_v);
    const int nblocks = (gp.nloc + lpb - 1) / lpb;
    const dim3 grid(nblocks), threads(lpb * 64);
    const int chunk = (gp.n[2] + (64 >> log2nvy) - 1) >> (6 - log2nvy);
    const int nvx_t = chunk <= 2 ? 2 : chunk <= 4 ? 4 : chunk <= 8 ? 8 : chunk <= 16 ? 16 : 32;
    const bool small = g.nd <= 512;
    if (map_dtype == GH_MAP_F16)
        return launch_cols_dt<GH_MAP_F16>(interp, small, nvx_t, grid, threads, lds, st, g, gp, lpb, log2nvy, maps, dec,
                                          block, excl, nexcl);
    if (map_dtype == GH_MAP_BF16)
        return launch_cols_dt<GH_MAP_BF16>(interp, small, nvx_t, grid, threads, lds, st, g, gp, lpb, log2nvy, maps,
                                           dec, block, excl, nexcl);
    return launch_cols_dt<GH_MAP_C64>(interp, small, nvx_t, grid, threads, lds, st, g, gp, lpb, log2nvy, maps, dec,
                                      block, excl, nexcl);
}

}  // namespace gh
