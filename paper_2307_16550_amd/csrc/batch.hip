// Batches of frames: the grid-hopping sweep (paper Sec. IV, eq. (7)) and the
// argmax of eqs. (5)-(6) over many frames of different shapes, each as one
// persistent launch that walks a device-resident frame-descriptor table.
//
// Sweep: a work unit is a tile of loc_tile consecutive locations of one frame
// (one by default), owned by one wave, which takes them in turn.  The
// wave keeps its FastGeo records and its receiver's Doppler table in a private
// LDS slice (sized for the batch's largest N_d), so the waves of a workgroup
// never synchronise with each other.  Lane (part, ivy) owns the vy column ivy
// over the vx rows [part*chunk, (part+1)*chunk) of the slab, for any Nvy <= 64
// (lanes beyond parts*Nvy evaluate discarded points).  The arithmetic per
// point is the column kernel's (same tables, same fixed-point coordinate with
// 2^32 = max(N_d, 512) bins), so the two agree bit for bit on shared shapes.
// Units are assigned statically, u = wave, wave + W, ... (W waves in the
// grid): every wave's share runs through all frames in order, which balances
// frames of different cost without a work counter (and so without anything to
// reset between runs: a captured graph replays as is).
#include "sweep_table.h"

namespace gh {
namespace {

constexpr int kMaxWaves = 4;
constexpr int kGeoF4 = (int)(sizeof(FastGeo) / sizeof(float4)) * kMaxRx;   // FastGeo records per wave slice

template <int INTERP, int NVX>
__global__ __launch_bounds__(64 * kMaxWaves) void sweep_batch(const FrameDesc* __restrict__ frames, int nf, int total,
                                                              int wave_f4, int loc_tile) {
    extern __shared__ float4 lds[];
    constexpr int kRun = INTERP ? 4 : 2;
    const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int wpb = blockDim.x >> 6;
    FastGeo* geo = reinterpret_cast<FastGeo*>(lds + (size_t)wid * wave_f4);
    float4* tabl = lds + (size_t)wid * wave_f4 + kGeoF4;
    const int stride = gridDim.x * wpb;
    int f = 0;
    for (int u = blockIdx.x * wpb + wid; u < total; u += stride) {
        while (f + 1 < nf && frames[f + 1].unit0[2] <= u) ++f;
        const FrameDesc* fd = frames + f;
        const int tile = u - fd->unit0[2];
        if (tile >= fd->nunit[2]) continue;   // not reached for a consistent table
        for (int loc = tile * loc_tile; loc < (tile + 1) * loc_tile && loc < fd->gp.nloc; ++loc) {
        const int k = fd->g.k, nd = fd->g.nd, log2nd = fd->g.log2_nd;
        const int log2p = log2nd > 9 ? log2nd : 9;   // 2^32 = 2^log2p Doppler bins
        const float sd = fd->g.sign_d;
        const int nvy = fd->nvy, chunk = fd->chunk, nvx = fd->gp.n[2];
        const int part = lane / nvy, ivy = lane - part * nvy;
        const int ivx0 = part * chunk;

        // geometry of (location, receiver q) by lane q; the previous unit's reads of
        // these records precede the writes in the wave's LDS order
        __builtin_amdgcn_wave_barrier();
        if (lane < k) geo[lane] = fast_geo<INTERP>(fd->g, fd->gp, loc, lane, 1.0 / (double)(1 << log2p), 8, 1.f);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();

        float acc[NVX];
#pragma unroll
        for (int j = 0; j < NVX; ++j) acc[j] = 0.f;
        const int runs = nd / kRun;
        const int rpl = (runs + 63) >> 6;
        const bool pipelined = (INTERP == 0) && rpl <= kPre;
        const char* maps = as_global(fd->maps);
        const size_t map_bytes = (size_t)__builtin_amdgcn_readfirstlane(fd->g.nr * nd) * 8;
        Prefetch pf;
        if (pipelined) table_prefetch<GH_MAP_C64>(pf, maps, geo[0], lane, rpl, runs, nd);
        const uint32_t bin_lo = (uint32_t)(32 - log2p), fsh = (uint32_t)(log2p - 9);
        for (int q = 0; q < k; ++q) {
            __builtin_amdgcn_wave_barrier();
            const char* mq = maps + (size_t)q * map_bytes;
            const FastGeo fb = geo[q];
            if (pipelined) table_store_prefetched(tabl, pf, fb, lane, rpl, runs, nd, sd);
            table_build<INTERP, GH_MAP_C64>(tabl, mq, fb, pipelined ? runs : lane, runs, nd, sd);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
            if (pipelined && q + 1 < k) table_prefetch<GH_MAP_C64>(pf, mq + map_bytes, geo[q + 1], lane, rpl, runs, nd);
            // the coordinate record is re-read here rather than kept live across the table build
            const FastGeo fg = geo[q];
            const uint32_t t = fg.t0 + (uint32_t)ivy * fg.ay + (uint32_t)ivx0 * fg.ax;
            // four table reads in flight (the single-frame kernel keeps eight for bilinear): this
            // keeps the bilinear 16-point column at 126 VGPRs, 4 waves per SIMD instead of 3
            eval_column<INTERP, NVX, 4>(acc, tabl, t, fg.ax, bin_lo, (uint32_t)log2nd, fsh, chunk);
        }

        // volume, then the location's maximum (ties to the lowest index)
        const int nv = fd->gp.nv;
        const bool on = part < fd->parts;
        int jmax = nvx - ivx0;
        if (jmax > chunk) jmax = chunk;
        if (!on) jmax = 0;
        float* dec = fd->dec ? as_global(fd->dec) : nullptr;
        if (dec) {
            float* dl = dec + (size_t)loc * nv + (size_t)ivx0 * nvy + ivy;
#pragma unroll
            for (int j = 0; j < NVX; ++j)
                if (j < jmax) dl[(size_t)j * nvy] = acc[j];
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
        int bi = bj < 0 ? 0x7fffffff : (ivx0 + bj) * nvy + ivy;
        wave_peak(bv, bi);
        if (lane == 0) {
            gh_peak p;
            p.value = bv;
            p.reserved = 0;
            p.index = (int64_t)loc * nv + (bi == 0x7fffffff ? 0 : bi);
            as_global(fd->block)[loc] = p;
        }
        }   // locations of the tile
    }
}

// Frame maxima: workgroup b reduces the block maxima of frames b, b + gridDim.x, ...
__global__ __launch_bounds__(1024) void peak_batch(const FrameDesc* __restrict__ frames, int nf,
                                                   gh_peak* __restrict__ argmax) {
    __shared__ float red_v[16];
    __shared__ long long red_i[16];
    for (int f = blockIdx.x; f < nf; f += gridDim.x) {
        float bv;
        long long bi;
        reduce_block_peaks(as_global(frames[f].block), frames[f].gp.nloc, bv, bi, red_v, red_i);
        if (threadIdx.x == 0) {
            gh_peak p;
            p.value = bv;
            p.reserved = 0;
            p.index = bi;
            argmax[f] = p;
        }
        __syncthreads();   // red_v / red_i are reused by the next frame
    }
}

template <int INTERP, int NVX>
hipError_t launch_nvx(int nf, int units, int wave_f4, int waves, int workgroups, int loc_tile,
                      const FrameDesc* frames, hipStream_t st) {
    const size_t lds = (size_t)waves * wave_f4 * sizeof(float4);
    hipLaunchKernelGGL((sweep_batch<INTERP, NVX>), dim3(workgroups), dim3(64 * waves), lds, st, frames, nf, units,
                       wave_f4, loc_tile);
    return hipGetLastError();
}

template <int INTERP>
hipError_t launch_interp(int nvx_t, int nf, int units, int wave_f4, int waves, int workgroups, int loc_tile,
                         const FrameDesc* frames, hipStream_t st) {
    switch (nvx_t) {
        case 4: return launch_nvx<INTERP, 4>(nf, units, wave_f4, waves, workgroups, loc_tile, frames, st);
        case 8: return launch_nvx<INTERP, 8>(nf, units, wave_f4, waves, workgroups, loc_tile, frames, st);
        case 16: return launch_nvx<INTERP, 16>(nf, units, wave_f4, waves, workgroups, loc_tile, frames, st);
        default: return launch_nvx<INTERP, 32>(nf, units, wave_f4, waves, workgroups, loc_tile, frames, st);
    }
}

template <int INTERP, int NVX>
int occupancy_nvx(int waves, size_t lds) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, sweep_batch<INTERP, NVX>, 64 * waves, lds) != hipSuccess)
        return 0;
    return per_cu;
}

template <int INTERP>
int occupancy_interp(int nvx_t, int waves, size_t lds) {
    switch (nvx_t) {
        case 4: return occupancy_nvx<INTERP, 4>(waves, lds);
        case 8: return occupancy_nvx<INTERP, 8>(waves, lds);
        case 16: return occupancy_nvx<INTERP, 16>(waves, lds);
        default: return occupancy_nvx<INTERP, 32>(waves, lds);
    }
}

}  // namespace

int sweep_batch_slice_f4(int interp, int nd_max) { return kGeoF4 + nd_max * (interp ? 2 : 1); }

// Smallest compiled column height holding `chunk_max` points; false beyond 32.
bool sweep_batch_nvx(int chunk_max, int& nvx_t) {
    if (chunk_max > 32) return false;
    nvx_t = chunk_max <= 4 ? 4 : chunk_max <= 8 ? 8 : chunk_max <= 16 ? 16 : 32;
    return true;
}

int sweep_batch_max_workgroups(int interp, int nvx_t, int waves, size_t lds) {
    const int per_cu = interp ? occupancy_interp<1>(nvx_t, waves, lds) : occupancy_interp<0>(nvx_t, waves, lds);
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t launch_sweep_batch(const FrameDesc* frames, int nf, int units, int interp, int nvx_t, int wave_f4,
                              int waves, int workgroups, int loc_tile, hipStream_t st) {
    const int need = (units + waves - 1) / waves;
    if (workgroups > need) workgroups = need;
    if (interp == GH_INTERP_BICUBIC)
        return launch_interp<1>(nvx_t, nf, units, wave_f4, waves, workgroups, loc_tile, frames, st);
    return launch_interp<0>(nvx_t, nf, units, wave_f4, waves, workgroups, loc_tile, frames, st);
}

hipError_t launch_peak_batch(const FrameDesc* frames, int nf, gh_peak* argmax, hipStream_t st) {
    hipLaunchKernelGGL(peak_batch, dim3(nf < 1024 ? nf : 1024), dim3(1024), 0, st, frames, nf, argmax);
    return hipGetLastError();
}

}  // namespace gh
