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
#include "sweep_table.h"

namespace gh {
namespace {

constexpr int kThreads = 256;

template <int INTERP, int MODE, int NVX, int DT>
__global__ __launch_bounds__(kThreads) void gh_sweep_columns(Geom g, GridP gp, int lpb, int log2nvy,
                                                            const char* __restrict__ maps, float* __restrict__ dec,
                                                            gh_peak* __restrict__ block,
                                                            const int64_t* __restrict__ excl, int nexcl) {
    extern __shared__ float4 lds[];
    constexpr int kEntry = INTERP ? 2 : 1;             // float4 per table entry
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
    const double inv = 1.0 / ((MODE == 0) ? 512.0 : (double)nd);
    for (int e = tid; e < lpb * g.k; e += blockDim.x) {
        const int q = e - (e / g.k) * g.k;
        geo[e] = fast_geo<INTERP>(g, gp, wg * lpb + e / g.k, q, inv, kEs, scale);
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
    const int rpl = (runs + 63) >> 6;
    const bool pipelined = (INTERP == 0) && rpl <= kPre;
    // uniform by construction: keeps the map base in scalar registers (g.nr is first read in the divergent loop above)
    const size_t map_bytes = (size_t)__builtin_amdgcn_readfirstlane(g.nr * nd) * kEs;
    Prefetch pf;
    if (pipelined) table_prefetch<DT>(pf, maps, geo[ll * g.k], lane, rpl, runs, nd);

    const uint32_t bin_lo = (MODE == 0) ? 23u : (uint32_t)(32 - log2nd);
    const uint32_t fsh = (MODE == 0) ? 0u : (uint32_t)(log2nd - 9);
    for (int q = 0; q < g.k; ++q) {
        // all lanes finished reading the previous receiver's table (in-order LDS per wave)
        __builtin_amdgcn_wave_barrier();
        const char* mq = maps + (size_t)q * map_bytes;
        const FastGeo fb = geo[ll * g.k + q];
        float4* tabl = tables + (size_t)ll * nd * kEntry;
        if (pipelined) table_store_prefetched(tabl, pf, fb, lane, rpl, runs, nd, sd);
        table_build<INTERP, DT>(tabl, mq, fb, pipelined ? runs : lane, runs, nd, sd);
        // the table is private to the wave: its LDS writes only have to land before the wave reads them
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        if (pipelined && q + 1 < g.k) table_prefetch<DT>(pf, mq + map_bytes, geo[ll * g.k + q + 1], lane, rpl, runs, nd);
        const FastGeo fg = geo[ll * g.k + q];
        const uint32_t t = fg.t0 + (uint32_t)ivy * fg.ay + (uint32_t)ivx0 * fg.ax;
        eval_column<INTERP, NVX>(acc, tabl, t, fg.ax, bin_lo, (uint32_t)log2nd, fsh, NVX);
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
    const int budget_kib = knob(GH_KNOB_SWEEP_LDS_KIB);   // test switch; default 40 KiB
    const size_t lds_budget = (budget_kib > 0 ? (size_t)budget_kib : 40) * 1024;
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
