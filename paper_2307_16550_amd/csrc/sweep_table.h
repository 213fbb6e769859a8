// Building blocks of the column sweep (paper Sec. IV, eq. (7)) shared by the
// single-frame kernel (sweep_fast.hip) and the persistent multi-frame kernel
// (batch.hip): the per-(location, receiver) geometry, the wave-private
// Doppler table of one receiver, and the evaluation of a column of points.
//
// Table entries, per Doppler segment [l, l+1] of the range-interpolated profile
// h (b = fraction of the Doppler coordinate):
//   bilinear: one float4 (e', d) with I = e' + (1 + b) d, d = h[l+1] - h[l], e' = h[l] - d
//   bicubic : two float4 (c0, c1), (c2, c3) with I = c0 + b c1 + b^2 c2 + b^3 c3 (Keys, a = -1/2)
// Indices past the period come from its start with the sign (-1)^(Mc-1)
// (centred maps).  Doppler coordinates are 32-bit fixed point with 2^32 = P
// bins, P = max(N_d, 512): the bin is the top log2 P bits masked to N_d - 1
// (exact since N_d divides P) and the top 23 bits of the fraction become the
// float 1 + b by insertion into the mantissa of 1.0.
#pragma once

#include "gh_internal.h"

namespace gh {

struct FastGeo {
    uint32_t row[4];   // byte offset of each range tap row (row index mod N_r, times N_d, times storage size)
    float w[4];        // range weights with the wrap sign and the storage scale folded in
    uint32_t t0;       // Doppler coordinate at (vx_lo, vy_lo)
    uint32_t ax;       // per vx step
    uint32_t ay;       // per vy step
    uint32_t pad;
};

// The bistatic range R and the sum w of the two unit vectors (eqs. (1)-(2)),
// FP64, with one reciprocal square root per leg instead of a square root and
// two divisions.
__device__ __forceinline__ void bistatic_rsq(const Geom& g, int q, double x, double y, double& r, double& wx,
                                             double& wy) {
    const double dx0 = x - g.tx[0], dy0 = y - g.tx[1];
    const double dx1 = x - g.rx[q][0], dy1 = y - g.rx[q][1];
    const double s0 = fma(dx0, dx0, dy0 * dy0), s1 = fma(dx1, dx1, dy1 * dy1);
    const double i0 = rsqrt_fp64(s0), i1 = rsqrt_fp64(s1);
    r = fma(s0, i0, s1 * i1);
    wx = fma(dx0, i0, dx1 * i1);
    wy = fma(dy0, i0, dy1 * i1);
}

// cycles_to_fixed without the 64-bit integer conversion: the rounded value
// lies in [0, 2^32], and 2^32 wraps to 0.
__device__ __forceinline__ uint32_t cycles_to_fixed32(double cyc) {
    const double s = fma(cyc - floor(cyc), 4294967296.0, 0.5);
    return s >= 4294967296.0 ? 0u : (uint32_t)s;
}

// Geometry of location `lc` (row-major over (x, y)) and receiver q; a zero
// record when lc is past the grid.  inv = 1 / P.
template <int INTERP>
__device__ __forceinline__ FastGeo fast_geo(const Geom& g, const GridP& gp, int lc, int q, double inv, int es,
                                            float scale) {
    constexpr int kTaps = INTERP ? 4 : 2;
    FastGeo fg;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        fg.row[u] = 0;
        fg.w[u] = 0.f;
    }
    fg.t0 = fg.ax = fg.ay = fg.pad = 0;
    if (lc < gp.nloc) {
        const int ix = lc / gp.n[1], iy = lc - ix * gp.n[1];
        double r, wx, wy;
        bistatic_rsq(g, q, gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], r, wx, wy);
        const double tr = g.kr * r;
        const double fl = floor(tr);
        const float a = (float)(tr - fl);
        const int i0 = (int)fl - (INTERP ? 1 : 0);
        float w[4];
        if (INTERP == 0) {
            w[0] = 1.f - a;
            w[1] = a;
            w[2] = w[3] = 0.f;
        } else {
            const float a2 = a * a, a3 = a2 * a;
            w[0] = -0.5f * a3 + a2 - 0.5f * a;
            w[1] = 1.5f * a3 - 2.5f * a2 + 1.f;
            w[2] = -1.5f * a3 + 2.f * a2 + 0.5f * a;
            w[3] = 0.5f * a3 - 0.5f * a2;
        }
#pragma unroll
        for (int u = 0; u < kTaps; ++u) {
            const int row = i0 + u;
            fg.row[u] = ((uint32_t)(row & (g.nr - 1)) << g.log2_nd) * (uint32_t)es;
            fg.w[u] = (((row >> g.log2_nr) & 1) ? g.sign_r * w[u] : w[u]) * scale;
        }
        fg.t0 = cycles_to_fixed32(g.kd * (wx * gp.lo[2] + wy * gp.lo[3]) * inv);
        fg.ax = cycles_to_fixed32(g.kd * wx * gp.step[2] * inv);
        fg.ay = cycles_to_fixed32(g.kd * wy * gp.step[3] * inv);
    }
    return fg;
}

__device__ __forceinline__ float2 wsum2(float w0, float2 a, float w1, float2 b) {
    return make_float2(fmaf(w1, b.x, w0 * a.x), fmaf(w1, b.y, w0 * a.y));
}

// Bilinear software pipeline: the map values of the next receiver's table,
// kPre runs of two entries per lane, held in registers while the current
// receiver's points are evaluated.
constexpr int kPre = 4;

struct Prefetch {
    float4 a[kPre], b[kPre];
    float2 a2[kPre], b2[kPre];
};

// fq by value: its row offsets are read from LDS once, not per prefetched run.
template <int DT>
__device__ __forceinline__ void table_prefetch(Prefetch& pf, const char* mq, const FastGeo fq, int lane, int rpl,
                                               int runs, int nd) {
    constexpr int kEs = map_elem_bytes(DT);
    const uint32_t r0 = fq.row[0], r1 = fq.row[1];
#pragma unroll
    for (int i = 0; i < kPre; ++i) {
        const int run = lane + 64 * i;
        if (i < rpl && run < runs) {
            const int l0 = run * 2;
            const uint32_t o0 = (uint32_t)l0 * kEs;
            const uint32_t ohi = (l0 + 2 == nd) ? 0u : o0 + 2u * kEs;
            pf.a[i] = map_ld2<DT>(mq, r0 + o0);
            pf.b[i] = map_ld2<DT>(mq, r1 + o0);
            pf.a2[i] = map_ld1<DT>(mq, r0 + ohi);
            pf.b2[i] = map_ld1<DT>(mq, r1 + ohi);
        }
    }
}

__device__ __forceinline__ void table_store_prefetched(float4* tab, const Prefetch& pf, const FastGeo& fb, int lane,
                                                       int rpl, int runs, int nd, float sd) {
    const float w0 = fb.w[0], w1 = fb.w[1];
#pragma unroll
    for (int i = 0; i < kPre; ++i) {
        const int run = lane + 64 * i;
        if (i < rpl && run < runs) {
            const int l0 = run * 2;
            const float shi = (l0 + 2 == nd) ? sd : 1.f;
            const float2 h0 = wsum2(w0, make_float2(pf.a[i].x, pf.a[i].y), w1, make_float2(pf.b[i].x, pf.b[i].y));
            const float2 h1 = wsum2(w0, make_float2(pf.a[i].z, pf.a[i].w), w1, make_float2(pf.b[i].z, pf.b[i].w));
            const float2 h2 = wsum2(w0 * shi, pf.a2[i], w1 * shi, pf.b2[i]);
            const float2 d0 = make_float2(h1.x - h0.x, h1.y - h0.y);
            const float2 d1 = make_float2(h2.x - h1.x, h2.y - h1.y);
            tab[l0] = make_float4(h0.x - d0.x, h0.y - d0.y, d0.x, d0.y);
            tab[l0 + 1] = make_float4(h1.x - d1.x, h1.y - d1.y, d1.x, d1.y);
        }
    }
}

// Bilinear tables of N_d = 128 NCH entries without guards: lane i builds the
// entry pairs (2 i + 128 c, 2 i + 1 + 128 c), c < NCH, from one vector load per
// map row and pair.  The profile value that follows a pair comes from lane
// i + 1 by a wave rotation (DPP); lane 63 takes lane 0's first value of the
// next chunk, or for the last chunk of the row's start with the sign of the
// next period.  Row offsets and weights are wave-uniform; per-chunk offsets
// are immediates.  The next receiver's values are prefetched into registers
// while the current table is evaluated.
template <int NCH>
struct PrefetchN {
    float4 a[NCH], b[NCH];
};

// o_lane: lane * 2 * (bytes per map value).
template <int DT, int NCH>
__device__ __forceinline__ void table_prefetch_n(PrefetchN<NCH>& pf, const char* mq, uint32_t r0, uint32_t r1,
                                                 uint32_t o_lane) {
    constexpr uint32_t kEs = map_elem_bytes(DT);
    const char* m0 = mq + r0;
    const char* m1 = mq + r1;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const uint32_t o0 = o_lane + (uint32_t)c * 128u * kEs;
        pf.a[c] = map_ld2<DT>(m0, o0);
        pf.b[c] = map_ld2<DT>(m1, o0);
    }
}

// Lane i receives lane (i + 1) mod 64's value (DPP wave_rol:1; all lanes active).
__device__ __forceinline__ float from_next_lane(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x134, 0xf, 0xf, false));
}

// tab: this lane's first pair (the wave's table + 2 lane entries).
template <int NCH>
__device__ __forceinline__ void table_store_n(float4* tab, const PrefetchN<NCH>& pf, float w0, float w1,
                                              bool last_lane, float sd) {
    float2 h0[NCH], h1[NCH], nx[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        h0[c] = wsum2(w0, make_float2(pf.a[c].x, pf.a[c].y), w1, make_float2(pf.b[c].x, pf.b[c].y));
        h1[c] = wsum2(w0, make_float2(pf.a[c].z, pf.a[c].w), w1, make_float2(pf.b[c].z, pf.b[c].w));
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c) nx[c] = make_float2(from_next_lane(h0[c].x), from_next_lane(h0[c].y));
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        const float2 wrap = (c == NCH - 1) ? make_float2(nx[0].x * sd, nx[0].y * sd) : nx[(c + 1) % NCH];
        const float2 h2 = last_lane ? wrap : nx[c];
        const float2 d0 = make_float2(h1[c].x - h0[c].x, h1[c].y - h0[c].y);
        const float2 d1 = make_float2(h2.x - h1[c].x, h2.y - h1[c].y);
        tab[128 * c] = make_float4(h0[c].x - d0.x, h0[c].y - d0.y, d0.x, d0.y);
        tab[128 * c + 1] = make_float4(h1[c].x - d1.x, h1[c].y - d1.y, d1.x, d1.y);
    }
}

// Table runs [run0, runs) in steps of 64 (kRun = 2 or 4 entries per run) built
// straight from the maps.
template <int INTERP, int DT>
__device__ __forceinline__ void table_build(float4* tabl, const char* mq, const FastGeo& fb, int run0, int runs, int nd,
                                            float sd) {
    constexpr int kEntry = INTERP ? 2 : 1;
    constexpr int kRun = INTERP ? 4 : 2;
    constexpr int kEs = map_elem_bytes(DT);
    for (int run = run0; run < runs; run += 64) {
        const int l0 = run * kRun;
        float4* tab = tabl + (size_t)l0 * kEntry;
        // profile values h[l0 - 1 .. l0 + 5]
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
}

// Accumulate |I|^2 of one receiver at the points t, t + ax, ... of a column
// (NVX points, evaluated in batches of LDS reads; batches starting at or
// beyond `jlim` are skipped, a wave-uniform bound).
template <int INTERP, int NVX, int WANT = (INTERP ? 4 : 8)>
__device__ __forceinline__ void eval_column(float (&acc)[NVX], const float4* tab, uint32_t t, uint32_t ax,
                                            uint32_t bin_lo, uint32_t log2nd, uint32_t fsh, int jlim) {
    constexpr int kEntry = INTERP ? 2 : 1;
    constexpr int kWant = WANT;                    // LDS reads kept in flight per column
    constexpr int kBatch = NVX < kWant ? NVX : kWant;
#pragma unroll
    for (int j0 = 0; j0 < NVX; j0 += kBatch) {
        if (j0 >= jlim) break;
        float4 e0[kBatch], e1[kBatch];
        float b1[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const uint32_t bin = __builtin_amdgcn_ubfe(t, bin_lo, log2nd);
            b1[u] = __uint_as_float(((t << fsh) & 0x007fffffu) | 0x3f800000u);   // 1 + fraction
            e0[u] = tab[bin * kEntry];
            if (INTERP) e1[u] = tab[bin * kEntry + 1];
            t += ax;
        }
        // issue the batch's reads before any of its arithmetic (the scheduler
        // would otherwise keep two in flight to save registers)
        __builtin_amdgcn_sched_barrier(0);
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

}  // namespace gh
