// Range-Doppler maps: per-receiver zero-padded 2D DFT (paper Sec. III and IV),
//   Z_q[i][l] = sum_m sum_s Y_q[m][s] exp(-j 2 pi (i (s - c_s)/N_r + l (m - c_m)/N_d)).
//
// Two passes through the output buffer, each an LDS Stockham FFT:
//   pass 1, range: one workgroup per (receiver, group of chirps).  Zero padding
//     by P is pruned: output i = P*q + p is the length-Ms FFT (index q) of the
//     chirp pre-twiddled by W_{N_r}^{p s}, so P short FFTs replace one long FFT
//     over a 3/4-zero input.  The spectrum of chirp m is parked, transposed, in
//     column m of the map rows (Z[q][i][m], m < Mc); a group of chirps per
//     workgroup makes those stores contiguous runs.
//   pass 2, Doppler: one workgroup per (receiver, group of range bins) reads the
//     first Mc entries of its rows, transforms them the same way along slow
//     time and overwrites the whole rows (each row is read and written by one
//     workgroup only, so the pass is in place).
// Centring multiplies output bin i by exp(j pi i (M-1)/N) (shift theorem).
#include "gh_internal.h"

namespace gh {
namespace {

constexpr int kThreads = 256;
constexpr int kLdsElems = 4096;   // complex values of the work buffer per workgroup (32 KiB)

// Twiddle table W_N^t = exp(-j 2 pi t / N), t < N, exact argument reduction.
__device__ void fill_twiddles(float2* tw, int n, int log2n) {
    for (int t = threadIdx.x; t < n; t += blockDim.x) {
        float s, c;
        // angle = -2 pi t / n = -pi * (2t/n); 2t/n is exact in float for n <= 2^24
        sincospif(__int2float_rn(2 * t) / __int2float_rn(n), &s, &c);
        tw[t] = make_float2(c, -s);
    }
}

// In-place forward FFTs of `nseq` contiguous sequences of length m = 2^log2m
// held in LDS buf[nseq][m].  Mixed radix-4/2 Stockham iterations; each stage
// reads all operands to registers, synchronises, then writes.  `tw` is the
// table of W_N^t with N = m * tw_stride.
__device__ void lds_fft(float2* buf, int nseq, int log2m, const float2* tw, int tw_stride) {
    const int m = 1 << log2m;
    const int total = nseq * m;
    int ns = 1;
    int remaining = log2m;
    while (remaining > 0) {
        const int radix = (remaining >= 2) ? 4 : 2;
        const int log2r = (radix == 4) ? 2 : 1;
        const int nbf = total >> log2r;          // butterflies in this stage
        const int per_seq = m >> log2r;
        // at most kLdsElems / 2 / kThreads = 8 butterflies per thread (static
        // register indexing: the loop bound is a compile-time constant)
        float2 v[8][4];
        int dst[8];
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int b = threadIdx.x + c * kThreads;
            if (b < nbf) {
                const int seq = b / per_seq;
                const int j = b - seq * per_seq;
                const int jm = j & (ns - 1);
                const float2* base = buf + seq * m;
                // twiddle exponent jm * r * m / (ns * radix), as an index into W_N
                const int tstep = (jm * (m / (ns * radix))) * tw_stride;
                const float2 a0 = base[j];
                const float2 a1 = cmul(base[j + per_seq], tw[tstep]);
                if (radix == 4) {
                    const float2 a2 = cmul(base[j + 2 * per_seq], tw[2 * tstep]);
                    const float2 a3 = cmul(base[j + 3 * per_seq], tw[3 * tstep]);
                    const float2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
                    const float2 s13 = cadd(a1, a3), d13 = csub(a1, a3);
                    const float2 jd13 = make_float2(d13.y, -d13.x);   // -j * d13
                    v[c][0] = cadd(s02, s13);
                    v[c][1] = cadd(d02, jd13);
                    v[c][2] = csub(s02, s13);
                    v[c][3] = csub(d02, jd13);
                } else {
                    v[c][0] = cadd(a0, a1);
                    v[c][1] = csub(a0, a1);
                    v[c][2] = v[c][1];
                    v[c][3] = v[c][1];
                }
                dst[c] = seq * m + (j - jm) * radix + jm;
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const int b = threadIdx.x + c * kThreads;
            if (b < nbf) {
                buf[dst[c]] = v[c][0];
                buf[dst[c] + ns] = v[c][1];
                if (radix == 4) {
                    buf[dst[c] + 2 * ns] = v[c][2];
                    buf[dst[c] + 3 * ns] = v[c][3];
                }
            }
        }
        __syncthreads();
        ns *= radix;
        remaining -= log2r;
    }
}

// exp(+j pi i (M-1) / N), exact reduction of i (M-1) modulo 2N.
__device__ __forceinline__ float2 centring_phase(int i, int mlen, int n) {
    const long long num = ((long long)i * (mlen - 1)) % (2LL * n);
    float s, c;
    sincospif((float)num / __int2float_rn(n), &s, &c);
    return make_float2(c, s);
}

// Pass 1: range FFT of `nch` chirps per workgroup.
__global__ __launch_bounds__(kThreads) void range_pass(Geom g, int nch, const float2* __restrict__ y,
                                                      float2* __restrict__ maps) {
    __shared__ float2 buf[kLdsElems];
    __shared__ float2 tw[4096];
    const int q = blockIdx.y;
    const int m0 = blockIdx.x * nch;
    const int ms = g.ms, nr = g.nr, pr = g.pr;
    fill_twiddles(tw, nr, g.log2_nr);
    __syncthreads();
    // pre-twiddled, pruned input: buf[c][p][s] = y[m0+c][s] * W_Nr^{p s}
    const int total = nch * nr;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int s = e & (ms - 1);
        const int p = (e >> g.log2_ms) % pr;
        const int c = e / nr;
        const float2 v = y[((size_t)q * g.mc + m0 + c) * ms + s];
        buf[e] = cmul(v, tw[p * s]);
    }
    __syncthreads();
    lds_fft(buf, nch * pr, g.log2_ms, tw, pr);
    // out bin i = pr*qq + p lives at buf[c][p][qq]; store transposed: Z[q][i][m0 + c]
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int c = e % nch;
        const int i = e / nch;
        const int p = i % pr, qq = i / pr;
        float2 v = buf[c * nr + p * ms + qq];
        if (g.centered) v = cmul(v, centring_phase(i, ms, nr));
        maps[((size_t)q * nr + i) * g.nd + m0 + c] = v;
    }
}

// Pass 2: Doppler FFT of `nrow` range bins per workgroup, in place.
__global__ __launch_bounds__(kThreads) void doppler_pass(Geom g, int nrow, float2* __restrict__ maps) {
    __shared__ float2 buf[kLdsElems];
    __shared__ float2 tw[4096];
    const int q = blockIdx.y;
    const int i0 = blockIdx.x * nrow;
    const int mc = g.mc, nd = g.nd, pd = g.pd;
    fill_twiddles(tw, nd, g.log2_nd);
    __syncthreads();
    const int total = nrow * nd;
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int m = e & (mc - 1);
        const int p = (e >> g.log2_mc) % pd;
        const int r = e / nd;
        const float2 v = maps[((size_t)q * g.nr + i0 + r) * nd + m];
        buf[e] = cmul(v, tw[p * m]);
    }
    __syncthreads();
    lds_fft(buf, nrow * pd, g.log2_mc, tw, pd);
    for (int e = threadIdx.x; e < total; e += blockDim.x) {
        const int l = e & (nd - 1);
        const int r = e >> g.log2_nd;
        const int p = l % pd, qq = l / pd;
        float2 v = buf[r * nd + p * mc + qq];
        if (g.centered) v = cmul(v, centring_phase(l, mc, nd));
        maps[((size_t)q * g.nr + i0 + r) * nd + l] = v;
    }
}

}  // namespace

hipError_t launch_rd_maps(const Geom& g, const float2* y, float2* maps, hipStream_t st) {
    int nch = kLdsElems / g.nr;
    if (nch > g.mc) nch = g.mc;
    int nrow = kLdsElems / g.nd;
    if (nrow > g.nr) nrow = g.nr;
    hipLaunchKernelGGL(range_pass, dim3(g.mc / nch, g.k), dim3(kThreads), 0, st, g, nch, y, maps);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(doppler_pass, dim3(g.nr / nrow, g.k), dim3(kThreads), 0, st, g, nrow, maps);
    return hipGetLastError();
}

}  // namespace gh
