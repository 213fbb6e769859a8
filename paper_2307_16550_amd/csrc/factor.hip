// Factorised decisions (paper Sec. III, eqs. (5)-(6); Sec. IV for grid
// hopping): the location first, from the energy of the per-chirp range
// correlations, then the velocity at the selected location.
//
//   E(x) = sum_q sum_m |g_q,x[m]|^2,  g_q,x[m] ~ <Y_q[m], a(f_r,q(x))>
//   V(v) = sum_q |sum_m g_q,x^[m] exp(-j 2 pi phi_q(v) m)|^2
//
// Direct: g is the range zoom G of the direct decision (matrix cores) and
// phi = f_d exactly.  Grid hopping: g is a range interpolation of the
// per-chirp range spectra (bilinear, Keys, or the polar rule: the three bins
// around the nearest one weighted by the circle through their atoms), and phi
// = round(t_d) / N_d, the nearest bin of the zero-padded FFT over chirps (the
// centring phase of that FFT has modulus one and drops out of |.|^2).
//
// Launches (nothing returns to the host in between):
//   1. location energy: one wave per location, lanes over chirps; the
//      geometry and range taps of receiver q come from lane q (FP64) by
//      shuffles; writes E and a block peak (E, location) per location;
//   2. the argmax of the block peaks into result[0] (ties to the lowest index);
//   3. velocity: 32 velocity points per workgroup, 8 lanes per point; per
//      receiver the workgroup puts g at the selected location in LDS, lane c
//      of a point sums the chirps m = c mod 8 of its Doppler correlation
//      (phases in 32-bit fixed point, an exact anchor every eight terms and a
//      rotation in between) and shuffles reduce the eight partial sums;
//      writes V and a peak per workgroup with the 4D index;
//   4. the argmax of those peaks into result[1].
#include "gh_internal.h"

namespace gh {
namespace {

constexpr int kLocWaves = 4;
constexpr int kVelThreads = 256;
constexpr int kVelLanes = 8;                              // lanes per velocity point (chirp classes mod 8)
constexpr int kVelPoints = kVelThreads / kVelLanes;       // velocity points per workgroup
constexpr int kRunF = 8;    // terms per exact phase anchor

struct RangeTaps {
    int row[4];     // range bin index within one period
    float w[4];     // weight with the wrap sign folded in (0 for unused taps)
};

// Taps of range coordinate tr (bins) for rule KIND (GH_INTERP_*).
template <int KIND>
__device__ __forceinline__ RangeTaps range_taps(const Geom& g, double tr, double theta) {
    double wd[4] = {0.0, 0.0, 0.0, 0.0};
    int i0;
    if (KIND == GH_INTERP_POLAR) {
        const double i = floor(tr + 0.5);
        const double tau = tr - i;
        const double a = (cos(theta * tau) - 1.0) / (2.0 * (1.0 - cos(theta)));
        const double b = sin(theta * tau) / (2.0 * sin(theta));
        i0 = (int)i - 1;
        wd[0] = -a - b;
        wd[1] = 1.0 + 2.0 * a;
        wd[2] = -a + b;
    } else if (KIND == GH_INTERP_BICUBIC) {
        const double fl = floor(tr);
        const double f = tr - fl, f2 = f * f, f3 = f2 * f;
        i0 = (int)fl - 1;
        wd[0] = -0.5 * f3 + f2 - 0.5 * f;
        wd[1] = 1.5 * f3 - 2.5 * f2 + 1.0;
        wd[2] = -1.5 * f3 + 2.0 * f2 + 0.5 * f;
        wd[3] = 0.5 * f3 - 0.5 * f2;
    } else {
        const double fl = floor(tr);
        i0 = (int)fl;
        wd[0] = 1.0 - (tr - fl);
        wd[1] = tr - fl;
    }
    RangeTaps t;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int row = i0 + u;
        t.row[u] = row & (g.nr - 1);
        t.w[u] = (float)((((row >> g.log2_nr) & 1) ? (double)g.sign_r : 1.0) * wd[u]);
    }
    return t;
}

template <int KIND>
constexpr int taps_of() {
    return KIND == GH_INTERP_BICUBIC ? 4 : KIND == GH_INTERP_POLAR ? 3 : 2;
}

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ void write_location(int loc, float e, float* loc_out, gh_peak* block) {
    if (loc_out) loc_out[loc] = e;
    gh_peak p;
    p.value = e;
    p.reserved = 0;
    p.index = loc;
    block[loc] = p;
}

// (5) by grid hopping: spectra complex64 [K][N_r][Mc].
template <int KIND>
__global__ __launch_bounds__(64 * kLocWaves) void location_energy_gh(Geom g, GridP gp, double theta,
                                                                     const float2* __restrict__ spec,
                                                                     float* __restrict__ loc_out,
                                                                     gh_peak* __restrict__ block) {
    constexpr int kTaps = taps_of<KIND>();
    const int lane = threadIdx.x & 63;
    const int loc = blockIdx.x * kLocWaves + (threadIdx.x >> 6);
    if (loc >= gp.nloc) return;   // whole waves
    const int ix = loc / gp.n[1], iy = loc - ix * gp.n[1];
    RangeTaps mine = {};
    if (lane < g.k) {
        double r, wx, wy;
        bistatic(g, lane, gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], r, wx, wy);
        mine = range_taps<KIND>(g, g.kr * r, theta);
    }
    const int mc = g.mc;
    float acc = 0.f;
    for (int q = 0; q < g.k; ++q) {
        const float2* sq = spec + (size_t)q * g.nr * mc;
        const float2* rows[kTaps];
        float w[kTaps];
#pragma unroll
        for (int u = 0; u < kTaps; ++u) {
            rows[u] = sq + (size_t)__shfl(mine.row[u], q, 64) * mc;
            w[u] = __shfl(mine.w[u], q, 64);
        }
        for (int m = lane; m < mc; m += 64) {
            float re = 0.f, im = 0.f;
#pragma unroll
            for (int u = 0; u < kTaps; ++u) {
                const float2 z = rows[u][m];
                re = fmaf(w[u], z.x, re);
                im = fmaf(w[u], z.y, im);
            }
            acc = fmaf(re, re, fmaf(im, im, acc));
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) write_location(loc, acc, loc_out, block);
}

// (5) directly: G float2 [K][Nloc][Mc] from the range zoom.
__global__ __launch_bounds__(64 * kLocWaves) void location_energy_direct(Geom g, GridP gp,
                                                                         const float2* __restrict__ G,
                                                                         float* __restrict__ loc_out,
                                                                         gh_peak* __restrict__ block) {
    const int lane = threadIdx.x & 63;
    const int loc = blockIdx.x * kLocWaves + (threadIdx.x >> 6);
    if (loc >= gp.nloc) return;
    const int mc = g.mc;
    float acc = 0.f;
    for (int q = 0; q < g.k; ++q) {
        const float2* gq = G + ((size_t)q * gp.nloc + loc) * mc;
        for (int m = lane; m < mc; m += 64) {
            const float2 z = gq[m];
            acc = fmaf(z.x, z.x, fmaf(z.y, z.y, acc));
        }
    }
    acc = wave_sum(acc);
    if (lane == 0) write_location(loc, acc, loc_out, block);
}

// (6) at the location selected in sel->index.  METHOD: GH_FACTOR_*.
template <int METHOD, int KIND>
__global__ __launch_bounds__(kVelThreads) void velocity_at_peak(Geom g, GridP gp, double theta,
                                                               const float2* __restrict__ input,
                                                               const gh_peak* __restrict__ sel,
                                                               float* __restrict__ vel_out,
                                                               gh_peak* __restrict__ vpeaks) {
    extern __shared__ float2 gvec[];   // [Mc]
    __shared__ float red_v[kVelThreads / 64];
    __shared__ int red_i[kVelThreads / 64];
    constexpr int kTaps = taps_of<KIND>();
    const int tid = threadIdx.x;
    const int cls = tid & (kVelLanes - 1);                 // this lane's chirps: m = cls mod 8
    // a selection outside the grid (every energy NaN: non-finite input) reads location 0
    const int loc = (sel->index >= 0 && sel->index < gp.nloc) ? (int)sel->index : 0;
    const int ix = loc / gp.n[1], iy = loc - ix * gp.n[1];
    const double x = gp.lo[0] + ix * gp.step[0], y = gp.lo[1] + iy * gp.step[1];
    const int v = blockIdx.x * kVelPoints + tid / kVelLanes;
    const bool live = v < gp.nv;
    const int ivx = live ? v / gp.n[3] : 0, ivy = live ? v - ivx * gp.n[3] : 0;
    const double vx = gp.lo[2] + ivx * gp.step[2], vy = gp.lo[3] + ivy * gp.step[3];
    const int mc = g.mc;
    float acc = 0.f;
    for (int q = 0; q < g.k; ++q) {
        double r, wx, wy;
        bistatic(g, q, x, y, r, wx, wy);
        if (METHOD == GH_FACTOR_DIRECT) {
            const float2* gq = input + ((size_t)q * gp.nloc + loc) * mc;
            for (int m = tid; m < mc; m += kVelThreads) gvec[m] = gq[m];
        } else {
            const RangeTaps t = range_taps<KIND>(g, g.kr * r, theta);
            const float2* sq = input + (size_t)q * g.nr * mc;
            for (int m = tid; m < mc; m += kVelThreads) {
                float re = 0.f, im = 0.f;
#pragma unroll
                for (int u = 0; u < kTaps; ++u) {
                    const float2 z = sq[(size_t)t.row[u] * mc + m];
                    re = fmaf(t.w[u], z.x, re);
                    im = fmaf(t.w[u], z.y, im);
                }
                gvec[m] = make_float2(re, im);
            }
        }
        __syncthreads();
        const double rate = wx * vx + wy * vy;
        uint32_t dph;   // phase per chirp, 2^32 = one cycle
        if (METHOD == GH_FACTOR_DIRECT) {
            dph = cycles_to_fixed(g.fd_per_mps * rate);
        } else {
            const long long l = (long long)floor(g.kd * rate + 0.5);   // nearest Doppler bin
            dph = (uint32_t)((unsigned long long)l << (32 - g.log2_nd));
        }
        const float2 rot = expm_fixed(dph * (uint32_t)kVelLanes);
        float cre = 0.f, cim = 0.f;
        for (int m0 = cls; m0 < mc; m0 += kVelLanes * kRunF) {
            float2 e = expm_fixed(dph * (uint32_t)m0);
#pragma unroll
            for (int u = 0; u < kRunF; ++u) {
                const int m = m0 + u * kVelLanes;
                if (m < mc) {
                    const float2 z = gvec[m];
                    cre = fmaf(z.x, e.x, fmaf(-z.y, e.y, cre));
                    cim = fmaf(z.x, e.y, fmaf(z.y, e.x, cim));
                }
                e = cmul(e, rot);
            }
        }
#pragma unroll
        for (int off = 1; off < kVelLanes; off <<= 1) {
            cre += __shfl_xor(cre, off, 64);
            cim += __shfl_xor(cim, off, 64);
        }
        acc = fmaf(cre, cre, fmaf(cim, cim, acc));
        __syncthreads();   // gvec is rewritten for the next receiver
    }
    if (live && cls == 0 && vel_out) vel_out[v] = acc;
    float bv = live ? acc : -INFINITY;
    int bi = live ? v : 0x7fffffff;
    wave_peak(bv, bi);
    if ((tid & 63) == 0) {
        red_v[tid >> 6] = bv;
        red_i[tid >> 6] = bi;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < kVelThreads / 64; ++w) peak_merge(bv, bi, red_v[w], red_i[w]);
        gh_peak p;
        p.value = bv;
        p.reserved = 0;
        p.index = (int64_t)loc * gp.nv + (bi == 0x7fffffff ? 0 : bi);
        vpeaks[blockIdx.x] = p;
    }
}

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

int velocity_groups(const GridP& gp) { return (gp.nv + kVelPoints - 1) / kVelPoints; }

template <int METHOD, int KIND>
void launch_velocity(const Geom& g, const GridP& gp, double theta, const float2* input, const gh_peak* sel,
                     float* vel, gh_peak* vpeaks, hipStream_t st) {
    hipLaunchKernelGGL((velocity_at_peak<METHOD, KIND>), dim3(velocity_groups(gp)), dim3(kVelThreads),
                       (size_t)g.mc * sizeof(float2), st, g, gp, theta, input, sel, vel, vpeaks);
}

template <int KIND>
void launch_gh_location(const Geom& g, const GridP& gp, double theta, const float2* spec, float* loc,
                        gh_peak* block, hipStream_t st) {
    hipLaunchKernelGGL(location_energy_gh<KIND>, dim3((gp.nloc + kLocWaves - 1) / kLocWaves), dim3(64 * kLocWaves), 0,
                       st, g, gp, theta, spec, loc, block);
}

}  // namespace

// Workspace: [G (direct only)] [block peaks, Nloc] [velocity peaks].
size_t factored_ws_bytes(const Geom& g, const GridP& gp, int method) {
    size_t b = align256((size_t)gp.nloc * sizeof(gh_peak)) + align256((size_t)velocity_groups(gp) * sizeof(gh_peak));
    if (method == GH_FACTOR_DIRECT) b += align256((size_t)g.k * gp.nloc * g.mc * sizeof(float2));
    return b;
}

hipError_t launch_factored(const Geom& g, const GridP& gp, int method, int range_interp, double polar_theta,
                           int gemm, const void* input, void* ws, float* loc, float* vel, gh_peak* result,
                           hipStream_t st) {
    char* w = static_cast<char*>(ws);
    float2* G = nullptr;
    if (method == GH_FACTOR_DIRECT) {
        G = reinterpret_cast<float2*>(w);
        w += align256((size_t)g.k * gp.nloc * g.mc * sizeof(float2));
    }
    gh_peak* block = reinterpret_cast<gh_peak*>(w);
    w += align256((size_t)gp.nloc * sizeof(gh_peak));
    gh_peak* vpeaks = reinterpret_cast<gh_peak*>(w);
    const dim3 lgrid((gp.nloc + kLocWaves - 1) / kLocWaves);
    hipError_t e;
    if (method == GH_FACTOR_DIRECT) {
        e = launch_direct_range(g, gp, static_cast<const float2*>(input), gemm, G, st);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(location_energy_direct, lgrid, dim3(64 * kLocWaves), 0, st, g, gp, G, loc, block);
    } else {
        const float2* spec = static_cast<const float2*>(input);
        if (range_interp == GH_INTERP_POLAR)
            launch_gh_location<GH_INTERP_POLAR>(g, gp, polar_theta, spec, loc, block, st);
        else if (range_interp == GH_INTERP_BICUBIC)
            launch_gh_location<GH_INTERP_BICUBIC>(g, gp, polar_theta, spec, loc, block, st);
        else
            launch_gh_location<GH_INTERP_BILINEAR>(g, gp, polar_theta, spec, loc, block, st);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = launch_peak_final(block, gp.nloc, result, nullptr, st)) != hipSuccess) return e;
    if (method == GH_FACTOR_DIRECT)
        launch_velocity<GH_FACTOR_DIRECT, GH_INTERP_BILINEAR>(g, gp, 0.0, G, result, vel, vpeaks, st);
    else if (range_interp == GH_INTERP_POLAR)
        launch_velocity<GH_FACTOR_GRID_HOPPING, GH_INTERP_POLAR>(g, gp, polar_theta, static_cast<const float2*>(input),
                                                                 result, vel, vpeaks, st);
    else if (range_interp == GH_INTERP_BICUBIC)
        launch_velocity<GH_FACTOR_GRID_HOPPING, GH_INTERP_BICUBIC>(g, gp, polar_theta,
                                                                   static_cast<const float2*>(input), result, vel,
                                                                   vpeaks, st);
    else
        launch_velocity<GH_FACTOR_GRID_HOPPING, GH_INTERP_BILINEAR>(g, gp, polar_theta,
                                                                    static_cast<const float2*>(input), result, vel,
                                                                    vpeaks, st);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_peak_final(vpeaks, velocity_groups(gp), result + 1, nullptr, st);
}

}  // namespace gh
