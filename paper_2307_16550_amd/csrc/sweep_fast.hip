// Grid-hopping sweep, column kernel (paper Sec. IV, eq. (7)): the variant used
// whenever the velocity slab has a power-of-two number of vy points (1..64),
// each thread's share of the vx axis is at most 32 points, and the
// per-location Doppler tables fit in LDS.
//
// Layout: a workgroup has `lpb` waves; each wave handles `lpw` locations in
// turn, one at a time (so one 8 KB table per wave for N_d = 512).  The
// geometry of a wave's lpw x K (location, receiver) pairs is computed once,
// one pair per lane, and kept in registers; pair p is read from lane p
// (readlane) when it is needed, so waves never wait for each other.
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
// LDS slice from vector loads straight from the maps, the next (location,
// receiver) pair's map values being prefetched into registers while the
// current table is evaluated: the range interpolation (2 or 4 map rows)
// collapses to a profile h[l], and each segment [l, l+1] stores the Doppler
// interpolant as a polynomial in the fraction:
//   bilinear: I = e' + (1 + b) d,        d = h[l+1] - h[l], e' = h[l] - d
//   bicubic : I = c0 + b c1 + b^2 c2 + b^3 c3   (Keys, a = -1/2)
// Bilinear tables of N_d = 128, 256 or 512 entries are built without guards:
// one 16-byte load per map row and entry pair, the following profile value
// from the next lane (DPP), immediate offsets.  Then every point reads one
// table entry (16 or 32 bytes of LDS), evaluates the polynomial and
// accumulates |I|^2 in a register.  The column loop is fully unrolled to a
// compile-time height NVX (points beyond the slab are evaluated on valid table
// entries and discarded) with its LDS reads issued in batches.  The volume and
// the block maximum (DPP row rotations, no LDS round trips) are written after
// the last receiver of each location.  Maps stored as 16-bit float pairs
// (Z / (Ms Mc)) are widened to FP32 in the table build, with the storage scale
// folded into the range weights.
#include "sweep_table.h"

namespace gh {
namespace {

constexpr int kThreads = 256;
constexpr int kMaxLpw = 4;          // locations per wave, at most
constexpr int kMinWaves = 16384;    // 64 waves per compute unit of a 256-unit device

// Lane p's value (p wave-uniform), in a scalar register.
__device__ __forceinline__ uint32_t lane_u32(uint32_t v, int p) { return (uint32_t)__builtin_amdgcn_readlane((int)v, p); }
__device__ __forceinline__ float lane_f32(float v, int p) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), p));
}

// The geometry record that lane p holds.
__device__ __forceinline__ FastGeo geo_of_lane(const FastGeo& mine, int p) {
    FastGeo f;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        f.row[u] = lane_u32(mine.row[u], p);
        f.w[u] = lane_f32(mine.w[u], p);
    }
    f.t0 = lane_u32(mine.t0, p);
    f.ax = lane_u32(mine.ax, p);
    f.ay = lane_u32(mine.ay, p);
    f.pad = 0;
    return f;
}

// NCH > 0: bilinear with N_d = 128 NCH (tables built without guards); 0: any shape.
// Each wave handles lpw locations in turn: location i of wave ll of workgroup
// wg is (wg lpw + i) lpb + ll, so at each step the waves of a workgroup hold
// lpb adjacent locations (their map rows largely shared in L1).
template <int INTERP, int MODE, int NVX, int DT, int NCH>
__global__ __launch_bounds__(kThreads) void gh_sweep_columns(Geom g, GridP gp, int lpb, int lpw, int log2nvy,
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

    const int tid = threadIdx.x;
    const int nvy = 1 << log2nvy;
    const int nvx = gp.n[2];
    // one location at a time per wave: lane = (part, ivy); part p owns vx rows [p*chunk, (p+1)*chunk)
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
    const int loc0 = wg * lpw * lpb + ll;

    // Geometry of the wave's lpw x K (location, receiver) pairs, held in
    // registers, one pair per lane (lane = i K + q); pair p is read from lane p
    // when it is needed.  The waves of a workgroup never wait for each other.
    const int npair = lpw * g.k;
    const double inv = 1.0 / ((MODE == 0) ? 512.0 : (double)nd);
    const int gi = lane / g.k;
    const FastGeo mine = fast_geo<INTERP>(g, gp, lane < npair ? loc0 + gi * lpb : gp.nloc, lane - gi * g.k, inv, kEs,
                                          scale);

    const float sd = g.sign_d;
    constexpr int kRun = INTERP ? 4 : 2;               // table entries per build run (2: lanes read contiguous float4)
    const int runs = nd / kRun;                        // table runs of this wave's location
    // Bilinear builds are software-pipelined: the map rows of the next
    // (location, receiver) pair are loaded into registers while the points of
    // the current one are evaluated.
    const int rpl = (runs + 63) >> 6;
    const bool pipelined = NCH == 0 && (INTERP == 0) && rpl <= kPre;
    // uniform by construction: keeps the map base in scalar registers (g.nr is first read in the divergent code above)
    const size_t map_bytes = (size_t)__builtin_amdgcn_readfirstlane(g.nr * nd) * kEs;
    const uint32_t bin_lo = (MODE == 0) ? 23u : (uint32_t)(32 - log2nd);
    const uint32_t fsh = (MODE == 0) ? 0u : (uint32_t)(log2nd - 9);
    const uint32_t o_lane = (uint32_t)lane * 2u * kEs;
    float4* tabl = tables + (size_t)ll * nd * kEntry;
    PrefetchN<NCH == 0 ? 1 : NCH> pfn;
    if constexpr (NCH > 0)
        table_prefetch_n<DT, NCH>(pfn, maps, lane_u32(mine.row[0], 0), lane_u32(mine.row[1], 0), o_lane);
    const int nv = gp.nv;
    const int jmax = (chunk < nvx - ivx0) ? chunk : nvx - ivx0;   // points of this thread inside the slab

    for (int i = 0; i < lpw; ++i) {
        const int loc = loc0 + i * lpb;
        if (loc >= gp.nloc) break;                     // wave-uniform: the rest lies past the grid
        float acc[NVX];
#pragma unroll
        for (int j = 0; j < NVX; ++j) acc[j] = 0.f;
        if constexpr (NCH > 0) {
            for (int q = 0; q < g.k; ++q) {
                __builtin_amdgcn_wave_barrier();
                const FastGeo fb = geo_of_lane(mine, i * g.k + q);
                const float w0 = fb.w[0], w1 = fb.w[1];
                table_store_n<NCH>(tabl + 2 * lane, pfn, w0, w1, lane == 63, sd);
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                // the next pair: receiver q + 1, or receiver 0 of the next location (a zero record past the grid)
                const int pn = i * g.k + q + 1;
                if (pn < npair) {
                    const int qn = (q + 1 < g.k) ? q + 1 : 0;
                    table_prefetch_n<DT, NCH>(pfn, maps + (size_t)qn * map_bytes, lane_u32(mine.row[0], pn),
                                              lane_u32(mine.row[1], pn), o_lane);
                }
                const uint32_t t = fb.t0 + (uint32_t)ivy * fb.ay + (uint32_t)ivx0 * fb.ax;
                eval_column<INTERP, NVX>(acc, tabl, t, fb.ax, bin_lo, (uint32_t)log2nd, fsh, NVX);
            }
        } else {
            Prefetch pf;
            if (pipelined) table_prefetch<DT>(pf, maps, geo_of_lane(mine, i * g.k), lane, rpl, runs, nd);
            for (int q = 0; q < g.k; ++q) {
                // all lanes finished reading the previous receiver's table (in-order LDS per wave)
                __builtin_amdgcn_wave_barrier();
                const char* mq = maps + (size_t)q * map_bytes;
                const FastGeo fb = geo_of_lane(mine, i * g.k + q);
                if (pipelined) table_store_prefetched(tabl, pf, fb, lane, rpl, runs, nd, sd);
                table_build<INTERP, DT>(tabl, mq, fb, pipelined ? runs : lane, runs, nd, sd);
                // the table is private to the wave: its LDS writes only have to land before the wave reads them
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
                if (pipelined && q + 1 < g.k)
                    table_prefetch<DT>(pf, mq + map_bytes, geo_of_lane(mine, i * g.k + q + 1), lane, rpl, runs, nd);
                const uint32_t t = fb.t0 + (uint32_t)ivy * fb.ay + (uint32_t)ivx0 * fb.ax;
                eval_column<INTERP, NVX>(acc, tabl, t, fb.ax, bin_lo, (uint32_t)log2nd, fsh, NVX);
            }
        }

        // volume, then the per-location maximum (ties to the lowest index)
        uint64_t skip = 0;      // bit j: point (ivx0 + j, ivy) is excluded from the maximum
        for (int e = 0; e < nexcl; ++e) {
            const int64_t d = excl[e] - (int64_t)loc * nv;
            if (d >= 0 && d < nv && (int)(d & (nvy - 1)) == ivy) {
                const int j = (int)(d >> log2nvy) - ivx0;
                if (j >= 0 && j < NVX) skip |= 1ull << j;
            }
        }
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
        wave_peak_rows(bv, bi);
        if (lane == 0) {
            gh_peak p;
            p.value = bv;
            p.reserved = 0;
            p.index = (int64_t)loc * nv + (bi == 0x7fffffff ? 0 : bi);
            block[loc] = p;
        }
    }
}

template <int INTERP, int MODE, int DT, int NCH>
hipError_t launch_cols(int nvx_t, dim3 grid, dim3 threads, size_t lds, hipStream_t st, const Geom& g,
                       const GridP& gp, int lpb, int lpw, int log2nvy, const char* maps, float* dec, gh_peak* block,
                       const int64_t* excl, int nexcl) {
    if (nvx_t == 2)
        hipLaunchKernelGGL((gh_sweep_columns<INTERP, MODE, 2, DT, NCH>), grid, threads, lds, st, g, gp, lpb, lpw,
                           log2nvy, maps, dec, block, excl, nexcl);
    else if (nvx_t == 4)
        hipLaunchKernelGGL((gh_sweep_columns<INTERP, MODE, 4, DT, NCH>), grid, threads, lds, st, g, gp, lpb, lpw,
                           log2nvy, maps, dec, block, excl, nexcl);
    else if (nvx_t == 8)
        hipLaunchKernelGGL((gh_sweep_columns<INTERP, MODE, 8, DT, NCH>), grid, threads, lds, st, g, gp, lpb, lpw,
                           log2nvy, maps, dec, block, excl, nexcl);
    else if (nvx_t == 16)
        hipLaunchKernelGGL((gh_sweep_columns<INTERP, MODE, 16, DT, NCH>), grid, threads, lds, st, g, gp, lpb, lpw,
                           log2nvy, maps, dec, block, excl, nexcl);
    else
        hipLaunchKernelGGL((gh_sweep_columns<INTERP, MODE, 32, DT, NCH>), grid, threads, lds, st, g, gp, lpb, lpw,
                           log2nvy, maps, dec, block, excl, nexcl);
    return hipGetLastError();
}

template <int DT>
hipError_t launch_cols_dt(int interp, bool small, int nvx_t, dim3 grid, dim3 threads, size_t lds, hipStream_t st,
                          const Geom& g, const GridP& gp, int lpb, int lpw, int log2nvy, const char* maps, float* dec,
                          gh_peak* block, const int64_t* excl, int nexcl) {
    if (interp == GH_INTERP_BICUBIC)
        return small ? launch_cols<1, 0, DT, 0>(nvx_t, grid, threads, lds, st, g, gp, lpb, lpw, log2nvy, maps, dec, block, excl, nexcl)
                     : launch_cols<1, 1, DT, 0>(nvx_t, grid, threads, lds, st, g, gp, lpb, lpw, log2nvy, maps, dec, block, excl, nexcl);
    if (!small)
        return launch_cols<0, 1, DT, 0>(nvx_t, grid, threads, lds, st, g, gp, lpb, lpw, log2nvy, maps, dec, block, excl, nexcl);
    if (g.nd == 512)
        return launch_cols<0, 0, DT, 4>(nvx_t, grid, threads, lds, st, g, gp, lpb, lpw, log2nvy, maps, dec, block, excl, nexcl);
    if (g.nd == 256)
        return launch_cols<0, 0, DT, 2>(nvx_t, grid, threads, lds, st, g, gp, lpb, lpw, log2nvy, maps, dec, block, excl, nexcl);
    if (g.nd == 128)
        return launch_cols<0, 0, DT, 1>(nvx_t, grid, threads, lds, st, g, gp, lpb, lpw, log2nvy, maps, dec, block, excl, nexcl);
    return launch_cols<0, 0, DT, 0>(nvx_t, grid, threads, lds, st, g, gp, lpb, lpw, log2nvy, maps, dec, block, excl, nexcl);
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
    const int cap = kThreads / 64;                   // one location at a time per wave
    const size_t per_wave = (size_t)g.nd * entry;
    const int fit = (int)(lds_budget / per_wave);
    lpb = cap < fit ? cap : fit;
    if (lpb < 1) return false;
    lds = (size_t)lpb * per_wave;
    return true;
}

// Locations per wave: up to kMaxLpw (and lpw K <= 64, one geometry pair per
// lane) while the grid still gives kMinWaves waves, enough to fill the device.
int sweep_columns_lpw(const Geom& g, const GridP& gp) {
    int lpw = kMaxLpw;
    while (lpw > 1 && (lpw * g.k > 64 || (long)gp.nloc < (long)lpw * kMinWaves)) lpw >>= 1;
    return lpw;
}

hipError_t launch_gh_sweep_columns(const Geom& g, const GridP& gp, int lpb, int log2nvy, size_t lds,
                                   const void* maps_v, int map_dtype, int interp, float* dec, gh_peak* block,
                                   const int64_t* excl, int nexcl, hipStream_t st) {
    const char* maps = static_cast<const char*>(maps_v);
    const int lpw = sweep_columns_lpw(g, gp);
    const int nblocks = (gp.nloc + lpb * lpw - 1) / (lpb * lpw);
    const dim3 grid(nblocks), threads(lpb * 64);
    const int chunk = (gp.n[2] + (64 >> log2nvy) - 1) >> (6 - log2nvy);
    const int nvx_t = chunk <= 2 ? 2 : chunk <= 4 ? 4 : chunk <= 8 ? 8 : chunk <= 16 ? 16 : 32;
    const bool small = g.nd <= 512;
    if (map_dtype == GH_MAP_F16)
        return launch_cols_dt<GH_MAP_F16>(interp, small, nvx_t, grid, threads, lds, st, g, gp, lpb, lpw, log2nvy, maps,
                                          dec, block, excl, nexcl);
    if (map_dtype == GH_MAP_BF16)
        return launch_cols_dt<GH_MAP_BF16>(interp, small, nvx_t, grid, threads, lds, st, g, gp, lpb, lpw, log2nvy,
                                           maps, dec, block, excl, nexcl);
    return launch_cols_dt<GH_MAP_C64>(interp, small, nvx_t, grid, threads, lds, st, g, gp, lpb, lpw, log2nvy, maps,
                                      dec, block, excl, nexcl);
}

}  // namespace gh
