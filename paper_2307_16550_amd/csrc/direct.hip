// Direct decision (paper Sec. I and III): exact scalar products of each
// receiver's frame with the atoms of eq. (3),
//   D_dir(x, v) = sum_q | sum_m sum_s Y_q[m][s] exp(-j 2 pi (f_r s + f_d m)) |^2,
// evaluated as two complex contractions per receiver on the matrix cores:
//   range zoom   G_q[x][m] = sum_s A[x][s] Y_q[m][s],   A[x][s] = exp(-j 2 pi f_r(x) s)
//                a [locations x Ms] x [Ms x Mc] product;
//   Doppler zoom c_q[ivx][ivy] = sum_m (G_q[x][m] Ex[ivx][m]) Ey[m][ivy]
//                per location a [Nvx x Mc] x [Mc x Nvy] product, because the
//                Doppler frequency is affine in the velocity indices,
//                f_d = f0 + ivx fx + ivy fy, so exp(-j 2 pi f_d m) factorises into
//                Ex[ivx][m] = exp(-j 2 pi (f0 + ivx fx) m) and Ey[m][ivy] = exp(-j 2 pi ivy fy m);
//   then |c_q|^2 summed over receivers, the slab write and the block maximum.
//
// Matrix-core mapping (64-lane wave, 16 x 16 output tile, FP32 accumulation):
//   lane = r + 16 g holds contraction indices k0 + 8 g + e (e = 0..7) of row r
//   of the left operand and of column r of the right operand.  BF16 issues
//   one 16x16x32 product per real part pairing; FP32 issues eight 16x16x4
//   products, the e-th taking element e of every lane (any assignment of
//   contraction indices to the k slots is valid if both operands share it).
//   The output element (i, j) sits in lane j + 16 (i / 4), slot i % 4.
// A complex product is four real ones:
//   Re C += Re A Re B - Im A Im B,  Im C += Re A Im B + Im A Re B.
// Atoms are generated in registers: one exact anchor per run of eight from a
// 32-bit fixed-point phase (the wrap modulo one cycle is integer overflow),
// then the recurrence e_{n+1} = e_n exp(-j 2 pi f).
#include "gh_internal.h"

namespace gh {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
constexpr int kThreads = 64 * kWaves;
constexpr int kRun = 8;     // contraction indices per lane per 32-wide step
constexpr int kNT = 4;      // 16-wide chirp tiles per wave in the range zoom

// exp(-j 2 pi f n) for n = n0 .. n0 + 7.
__device__ __forceinline__ void atom_run(uint32_t f, uint32_t n0, float2 ratio, float2 (&e)[kRun]) {
    e[0] = expm_fixed(f * n0);
#pragma unroll
    for (int i = 1; i < kRun; ++i) e[i] = cmul(e[i - 1], ratio);
}

__device__ __forceinline__ f32x4 zero4() { return f32x4{0.f, 0.f, 0.f, 0.f}; }

// C += A B for complex operands held as kRun values per lane (layout above).
template <bool BF16>
__device__ __forceinline__ void mfma_complex(const float2 (&a)[kRun], const float2 (&b)[kRun], f32x4& cre,
                                             f32x4& cim) {
    if constexpr (BF16) {
        bf16x8 ar, ai, nai, br, bi;
#pragma unroll
        for (int e = 0; e < kRun; ++e) {
            ar[e] = (__bf16)a[e].x;
            ai[e] = (__bf16)a[e].y;
            nai[e] = (__bf16)(-a[e].y);
            br[e] = (__bf16)b[e].x;
            bi[e] = (__bf16)b[e].y;
        }
        cre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, br, cre, 0, 0, 0);
        cre = __builtin_amdgcn_mfma_f32_16x16x32_bf16(nai, bi, cre, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ar, bi, cim, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ai, br, cim, 0, 0, 0);
    } else {
#pragma unroll
        for (int e = 0; e < kRun; ++e) {
            cre = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e].x, b[e].x, cre, 0, 0, 0);
            cre = __builtin_amdgcn_mfma_f32_16x16x4f32(-a[e].y, b[e].y, cre, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e].x, b[e].y, cim, 0, 0, 0);
            cim = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e].y, b[e].x, cim, 0, 0, 0);
        }
    }
}

__device__ __forceinline__ void load_run(const float2* __restrict__ p, float2 (&v)[kRun]) {
    const float4* p4 = reinterpret_cast<const float4*>(p);
#pragma unroll
    for (int i = 0; i < kRun / 2; ++i) {
        const float4 t = p4[i];
        v[2 * i] = make_float2(t.x, t.y);
        v[2 * i + 1] = make_float2(t.z, t.w);
    }
}

// Range zoom.  Grid (ceil(Nloc / 64), ceil(Mc / 64), K); wave w of a
// workgroup owns 16 locations and 64 chirps of receiver blockIdx.z.
template <bool BF16>
__global__ __launch_bounds__(kThreads) void direct_range_zoom(Geom g, GridP gp, const float2* __restrict__ y,
                                                             float2* __restrict__ gws) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int seg = lane >> 4;
    const int q = blockIdx.z;
    const int loc0 = (blockIdx.x * kWaves + (threadIdx.x >> 6)) * 16;
    const int m0 = blockIdx.y * (16 * kNT);
    const int ms = g.ms, mc = g.mc;

    uint32_t fr = 0;
    if (loc0 + r < gp.nloc) {
        const int loc = loc0 + r;
        const int ix = loc / gp.n[1], iy = loc - ix * gp.n[1];
        double rr, wx, wy;
        bistatic(g, q, gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], rr, wx, wy);
        fr = cycles_to_fixed(g.fr_per_m * rr);
    }
    const float2 ratio = expm_fixed(fr);

    f32x4 cre[kNT], cim[kNT];
#pragma unroll
    for (int t = 0; t < kNT; ++t) cre[t] = cim[t] = zero4();

    const float2* yq = y + (size_t)q * mc * ms;
    for (int s0 = 0; s0 < ms; s0 += 32) {
        const int sb = s0 + seg * kRun;
        const bool live = sb < ms;   // Ms is a power of two >= 8: a run is all in or all out
        float2 a[kRun];
        atom_run(fr, (uint32_t)sb, ratio, a);
        if (!live) {
#pragma unroll
            for (int e = 0; e < kRun; ++e) a[e] = make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int t = 0; t < kNT; ++t) {
            const int m = m0 + t * 16 + r;
            float2 b[kRun];
            if (live && m < mc) {
                load_run(yq + (size_t)m * ms + sb, b);
            } else {
#pragma unroll
                for (int e = 0; e < kRun; ++e) b[e] = make_float2(0.f, 0.f);
            }
            mfma_complex<BF16>(a, b, cre[t], cim[t]);
        }
    }
#pragma unroll
    for (int t = 0; t < kNT; ++t) {
        const int m = m0 + t * 16 + r;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int loc = loc0 + 4 * seg + e;
            if (loc < gp.nloc && m < mc) gws[((size_t)q * gp.nloc + loc) * mc + m] = make_float2(cre[t][e], cim[t][e]);
        }
    }
}

// Range zoom with BF16 operands: as below, but the four waves share the frame
// operand: each 32-sample step of the 64 chirps is staged once in LDS
// (double-buffered, rows padded to an odd number of 16-byte words so the
// operand reads do not conflict) instead of being read from L2 by every wave.
// BF16 products are cheap enough that those L2 reads bound the kernel (71 ->
// 53 us for the BF16 direct decision of the paper-scale subgrid); in FP32 the
// staging gains 2 us and its 35 KB of LDS cost more beside other kernels.
constexpr int kYRows = 16 * kNT;                 // chirps per workgroup
constexpr int kYRow4 = 32 / 2 + 1;              // float4 per staged row: 32 samples + padding

__global__ __launch_bounds__(kThreads) void direct_range_zoom_bf16(Geom g, GridP gp, const float2* __restrict__ y,
                                                                  float2* __restrict__ gws) {
    constexpr bool BF16 = true;
    __shared__ float4 ytile[2][kYRows][kYRow4];
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int seg = lane >> 4;
    const int q = blockIdx.z;
    const int loc0 = (blockIdx.x * kWaves + (threadIdx.x >> 6)) * 16;
    const int m0 = blockIdx.y * kYRows;
    const int ms = g.ms, mc = g.mc;

    uint32_t fr = 0;
    if (loc0 + r < gp.nloc) {
        const int loc = loc0 + r;
        const int ix = loc / gp.n[1], iy = loc - ix * gp.n[1];
        double rr, wx, wy;
        bistatic(g, q, gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], rr, wx, wy);
        fr = cycles_to_fixed(g.fr_per_m * rr);
    }
    const float2 ratio = expm_fixed(fr);

    f32x4 cre[kNT], cim[kNT];
#pragma unroll
    for (int t = 0; t < kNT; ++t) cre[t] = cim[t] = zero4();

    // staging: 64 rows x 16 float4 (32 samples) per step, four float4 per thread
    const float4* yq4 = reinterpret_cast<const float4*>(y + (size_t)q * mc * ms);
    constexpr int kPer = kYRows * 16 / kThreads;
    float4 stage[kPer];
    auto load_step = [&](int s0) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int idx = threadIdx.x + i * kThreads;
            const int row = idx >> 4, c4 = idx & 15;
            const int m = m0 + row, s = s0 + 2 * c4;
            stage[i] = (m < mc && s < ms) ? yq4[((size_t)m * ms + s) >> 1] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto store_step = [&](int buf) {
#pragma unroll
        for (int i = 0; i < kPer; ++i) {
            const int idx = threadIdx.x + i * kThreads;
            ytile[buf][idx >> 4][idx & 15] = stage[i];
        }
    };
    load_step(0);
    store_step(0);
    __syncthreads();
    int buf = 0;
    for (int s0 = 0; s0 < ms; s0 += 32) {
        const bool more = s0 + 32 < ms;
        if (more) load_step(s0 + 32);
        const int sb = s0 + seg * kRun;
        const bool live = sb < ms;   // Ms is a power of two >= 8: a run is all in or all out
        float2 a[kRun];
        atom_run(fr, (uint32_t)sb, ratio, a);
        if (!live) {
#pragma unroll
            for (int e = 0; e < kRun; ++e) a[e] = make_float2(0.f, 0.f);
        }
#pragma unroll
        for (int t = 0; t < kNT; ++t) {
            float2 b[kRun];
            const float4* row = ytile[buf][t * 16 + r] + seg * (kRun / 2);
#pragma unroll
            for (int i = 0; i < kRun / 2; ++i) {
                const float4 v = row[i];
                b[2 * i] = make_float2(v.x, v.y);
                b[2 * i + 1] = make_float2(v.z, v.w);
            }
            mfma_complex<BF16>(a, b, cre[t], cim[t]);
        }
        if (more) store_step(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int t = 0; t < kNT; ++t) {
        const int m = m0 + t * 16 + r;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int loc = loc0 + 4 * seg + e;
            if (loc < gp.nloc && m < mc) gws[((size_t)q * gp.nloc + loc) * mc + m] = make_float2(cre[t][e], cim[t][e]);
        }
    }
}

// Doppler zoom.  One wave per location; it walks the 16 x 16 tiles of the
// velocity slab, sums |c_q|^2 over receivers, writes the slab and reduces the
// block maximum (ties to the lowest index), skipping excluded cells.
template <bool BF16>
__global__ __launch_bounds__(kThreads) void direct_doppler_zoom(Geom g, GridP gp, const float2* __restrict__ gws,
                                                               float* __restrict__ dec, gh_peak* __restrict__ block,
                                                               const int64_t* __restrict__ excl, int nexcl) {
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int seg = lane >> 4;
    const int loc = blockIdx.x * kWaves + (threadIdx.x >> 6);
    if (loc >= gp.nloc) return;
    const int ix = loc / gp.n[1], iy = loc - ix * gp.n[1];
    const int nvx = gp.n[2], nvy = gp.n[3], nv = gp.nv, mc = g.mc;

    // Doppler frequency of receiver `lane` at the slab origin and its steps per vx / vy index
    uint32_t f0l = 0, fxl = 0, fyl = 0;
    if (lane < g.k) {
        double rr, wx, wy;
        bistatic(g, lane, gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], rr, wx, wy);
        f0l = cycles_to_fixed(g.fd_per_mps * (wx * gp.lo[2] + wy * gp.lo[3]));
        fxl = cycles_to_fixed_step(g.fd_per_mps * wx * gp.step[2]);
        fyl = cycles_to_fixed_step(g.fd_per_mps * wy * gp.step[3]);
    }

    const int tiles_y = (nvy + 15) >> 4;
    const int ntiles = ((nvx + 15) >> 4) * tiles_y;
    const int64_t base = (int64_t)loc * nv;
    float best_v = -INFINITY;
    int best_i = 0x7fffffff;
    for (int tile = 0; tile < ntiles; ++tile) {
        const int tx = tile / tiles_y, ty = tile - tx * tiles_y;
        f32x4 dsum = zero4();
        for (int q = 0; q < g.k; ++q) {
            const uint32_t f0 = (uint32_t)__shfl((int)f0l, q, 64);
            const uint32_t fx = (uint32_t)__shfl((int)fxl, q, 64);
            const uint32_t fy = (uint32_t)__shfl((int)fyl, q, 64);
            const uint32_t fa = f0 + (uint32_t)(tx * 16 + r) * fx;   // row ivx = 16 tx + r of Ex
            const uint32_t fb = (uint32_t)(ty * 16 + r) * fy;        // column ivy = 16 ty + r of Ey
            const float2 ra = expm_fixed(fa), rb = expm_fixed(fb);
            const float2* gq = gws + ((size_t)q * gp.nloc + loc) * mc;
            f32x4 cre = zero4(), cim = zero4();
            for (int k0 = 0; k0 < mc; k0 += 32) {
                const int mb = k0 + seg * kRun;
                float2 a[kRun], b[kRun];
                if (mb < mc) {   // Mc is a power of two >= 8: a run is all in or all out
                    float2 gv[kRun];
                    load_run(gq + mb, gv);
                    atom_run(fa, (uint32_t)mb, ra, a);
                    atom_run(fb, (uint32_t)mb, rb, b);
#pragma unroll
                    for (int e = 0; e < kRun; ++e) a[e] = cmul(gv[e], a[e]);
                } else {
#pragma unroll
                    for (int e = 0; e < kRun; ++e) a[e] = b[e] = make_float2(0.f, 0.f);
                }
                mfma_complex<BF16>(a, b, cre, cim);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) dsum[e] = fmaf(cre[e], cre[e], fmaf(cim[e], cim[e], dsum[e]));
        }
        const int ivy = ty * 16 + r;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int ivx = tx * 16 + 4 * seg + e;
            if (ivx < nvx && ivy < nvy) {
                const int v = ivx * nvy + ivy;
                if (dec) dec[base + v] = dsum[e];
                bool skip = false;
                for (int i = 0; i < nexcl; ++i) skip |= (excl[i] == base + v);
                if (!skip) peak_merge(best_v, best_i, dsum[e], v);
            }
        }
    }
    wave_peak(best_v, best_i);
    if (lane == 0) {
        gh_peak p;
        p.value = best_v;
        p.reserved = 0;
        p.index = base + (best_i == 0x7fffffff ? 0 : best_i);
        block[loc] = p;
    }
}

}  // namespace

size_t direct_ws_bytes(const Geom& g, const GridP& gp, int /*gemm*/) {
    return (size_t)g.k * gp.nloc * g.mc * sizeof(float2);
}

hipError_t launch_direct_range(const Geom& g, const GridP& gp, const float2* y, int gemm, float2* G, hipStream_t st) {
    const dim3 g1((gp.nloc + 16 * kWaves - 1) / (16 * kWaves), (g.mc + 16 * kNT - 1) / (16 * kNT), g.k);
    if (gemm == GH_GEMM_BF16)
        hipLaunchKernelGGL(direct_range_zoom_bf16, g1, dim3(kThreads), 0, st, g, gp, y, G);
    else
        hipLaunchKernelGGL(direct_range_zoom<false>, g1, dim3(kThreads), 0, st, g, gp, y, G);
    return hipGetLastError();
}

hipError_t launch_direct(const Geom& g, const GridP& gp, const float2* y, int gemm, void* ws, float* dec,
                         gh_peak* block, const int64_t* excl, int nexcl, hipStream_t st) {
    float2* gws = static_cast<float2*>(ws);
    const dim3 g1((gp.nloc + 16 * kWaves - 1) / (16 * kWaves), (g.mc + 16 * kNT - 1) / (16 * kNT), g.k);
    const dim3 g2((gp.nloc + kWaves - 1) / kWaves);
    if (gemm == GH_GEMM_BF16) {
        hipLaunchKernelGGL(direct_range_zoom_bf16, g1, dim3(kThreads), 0, st, g, gp, y, gws);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(direct_doppler_zoom<true>, g2, dim3(kThreads), 0, st, g, gp, gws, dec, block, excl, nexcl);
    } else {
        hipLaunchKernelGGL(direct_range_zoom<false>, g1, dim3(kThreads), 0, st, g, gp, y, gws);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(direct_doppler_zoom<false>, g2, dim3(kThreads), 0, st, g, gp, gws, dec, block, excl,
                           nexcl);
    }
    return hipGetLastError();
}

}  // namespace gh
