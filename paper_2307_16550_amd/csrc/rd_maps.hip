// Range-Doppler maps: per-receiver zero-padded 2D DFT (paper Sec. III and IV),
//   Z_q[i][l] = sum_m sum_s Y_q[m][s] exp(-j 2 pi (i (s - c_s)/N_r + l (m - c_m)/N_d)),
// with c = (M - 1)/2 for centred maps and c = 0 otherwise.
//
// Zero padding by P is pruned on both axes: output bin P k + p of a length-N
// transform (N = P M) of a length-M sequence x is
//   e^{j 2 pi (P k + p) c / N} sum_s x[s] W_N^{p s} W_M^{k s}
//   = cen[k] * FFT_M( x[s] * pre_p[s] )[k],
//   pre_p[s] = exp(-j pi p (2 s - 2 c) / N),   cen[k] = exp(j 2 pi k c / M),
// so P short FFTs on pre-twiddled inputs replace one long FFT over a mostly
// zero input, and the centring costs one table product per element.  Tables
// are built per workgroup with exact integer argument reduction.
//
// Two passes through the output buffer, each an LDS Stockham FFT (radix 4/2):
//   pass 1, range: one workgroup per (receiver, sub-transform p, group of G
//     chirps); the spectra are parked, transposed, in columns m < Mc of the map
//     rows (Z[q][P k + p][m]), G consecutive chirps per store run.
//   pass 2, Doppler: one workgroup per (receiver, group of range rows) reads the
//     first Mc entries of its rows, applies the P sub-transforms and overwrites
//     the whole rows (each row is read and written by one workgroup only) in
//     the storage type: complex64, or 16-bit pairs holding Z / (Ms Mc) (a half
//     row of N_d 4-byte entries still holds the Mc 8-byte parked values when
//     P_d >= 2).
// LDS sequences are padded to an odd stride so the transposed reads of the
// store phase do not conflict.  For single frames whose transforms fit one
// wave (Ms <= 512, P_d Mc <= 512, or twice that with P_d >= 2), each wave
// owns one chirp (pass 1) or one row, or half of a row's P_d sub-transforms
// when P_d >= 2 (pass 2), and runs its stages without workgroup barriers
// (range_pass_w, doppler_pass_w); batches and larger frames use the
// workgroup-wide passes.
#include "gh_internal.h"

namespace gh {
namespace {

constexpr int kThreads = 512;

// Complex product with the fused multiply-adds spelled out, so that every pass
// below (workgroup-wide or one transform per wave, single frames or batches)
// rounds the same way and their maps agree bit for bit.
__device__ __forceinline__ float2 cmulf(float2 a, float2 b) {
    return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
constexpr int kBuf = 4096;        // complex values of FFT work per workgroup
constexpr int kBfly = kBuf / 2 / kThreads;   // butterflies per thread and stage, at most

// exp(-j pi num / den) with the numerator reduced exactly modulo 2 den; den is
// a power of two (every transform length here is), so the reduction is a mask
// (two's complement gives the non-negative residue for negative num too).
__device__ __forceinline__ float2 expm_pi(long long num, int den) {
    const long long r = num & (2LL * den - 1);
    float s, c;
    sincospif((float)r / (float)den, &s, &c);
    return make_float2(c, -s);
}

// pre[s] = exp(-j pi p (2 s - c2) / N) for s < M (c2 = M - 1 when centred, else 0;
// for every p < np when all_p, none when np == 0), tw[t] = W_M^t for t < M,
// cen[k] = exp(+j pi k c2 / M) for k < M.
__device__ void fill_tables(float2* pre, float2* tw, float2* cen, int p, int m, int n, int centered,
                            bool all_p, int np) {
    const int c2 = centered ? m - 1 : 0;
    const int npre = all_p ? np * m : (np > 0 ? m : 0);
    for (int t = threadIdx.x; t < npre; t += blockDim.x) {
        const int pp = all_p ? t / m : p;
        const int s = all_p ? t - pp * m : t;
        pre[t] = expm_pi((long long)pp * (2LL * s - c2), n);
    }
    for (int t = threadIdx.x; t < m; t += blockDim.x) {
        tw[t] = expm_pi(2LL * t, m);
        const float2 e = expm_pi((long long)t * c2, m);
        cen[t] = make_float2(e.x, -e.y);
    }
}

// In-place forward FFTs of `nseq` sequences of length m = 2^log2m, sequence j at
// buf + j * stride.  Mixed radix-4/2 Stockham iterations; each stage reads all
// operands to registers, synchronises, then writes.  tw[t] = W_m^t.
__device__ void lds_fft(float2* buf, int nseq, int stride, int log2m, const float2* tw) {
    const int m = 1 << log2m;
    int ns = 1, log2ns = 0;
    int remaining = log2m;
    while (remaining > 0) {
        const int log2r = (remaining >= 2) ? 2 : 1;
        const int per_seq = m >> log2r;               // butterflies per sequence
        const int log2ps = log2m - log2r;
        const int nbf = nseq << log2ps;
        // at most kBfly butterflies per thread (static register indexing)
        float2 v[kBfly][4];
        int dst[kBfly];
#pragma unroll
        for (int c = 0; c < kBfly; ++c) {
            const int b = threadIdx.x + c * kThreads;
            if (b < nbf) {
                const int seq = b >> log2ps;
                const int j = b & (per_seq - 1);
                const int jm = j & (ns - 1);
                const float2* base = buf + seq * stride;
                // twiddle exponent jm * m / (ns * radix)
                const int tstep = jm << (log2m - log2ns - log2r);
                const float2 a0 = base[j];
                const float2 a1 = cmulf(base[j + per_seq], tw[tstep]);
                if (log2r == 2) {
                    const float2 a2 = cmulf(base[j + 2 * per_seq], tw[2 * tstep]);
                    const float2 a3 = cmulf(base[j + 3 * per_seq], tw[3 * tstep]);
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
                dst[c] = seq * stride + ((j - jm) << log2r) + jm;
            }
        }
        __syncthreads();
#pragma unroll
        for (int c = 0; c < kBfly; ++c) {
            const int b = threadIdx.x + c * kThreads;
            if (b < nbf) {
                buf[dst[c]] = v[c][0];
                buf[dst[c] + ns] = v[c][1];
                if (log2r == 2) {
                    buf[dst[c] + 2 * ns] = v[c][2];
                    buf[dst[c] + 3 * ns] = v[c][3];
                }
            }
        }
        __syncthreads();
        ns <<= log2r;
        log2ns += log2r;
        remaining -= log2r;
    }
}

// The same FFTs run by one wave on sequences of its own (at most kWavePts
// complex values in all): with no other wave touching them, the stages need
// no workgroup barrier; a wave's LDS instructions complete in issue order, so
// every lane's reads of a stage precede every lane's writes of it.  (At 1024
// points per wave the register arrays cut the occupancy, and the maps of a
// K = 8, Ms = 512, Mc = 256 frame took 130 us against 97 us with the
// workgroup-wide passes.)
constexpr int kWavePts = 512;

template <int NP>   // at most NP points per wave
__device__ void wave_fft(float2* buf, int nseq, int stride, int log2m, const float2* tw) {
    constexpr int kWaveBfly = NP / 2 / 64;
    const int lane = threadIdx.x & 63;
    const int m = 1 << log2m;
    int ns = 1, log2ns = 0;
    int remaining = log2m;
    while (remaining > 0) {
        const int log2r = (remaining >= 2) ? 2 : 1;
        const int per_seq = m >> log2r;
        const int log2ps = log2m - log2r;
        const int nbf = nseq << log2ps;
        float2 v[kWaveBfly][4];
        int dst[kWaveBfly];
#pragma unroll
        for (int c = 0; c < kWaveBfly; ++c) {
            const int b = lane + c * 64;
            if (b < nbf) {
                const int seq = b >> log2ps;
                const int j = b & (per_seq - 1);
                const int jm = j & (ns - 1);
                const float2* base = buf + seq * stride;
                const int tstep = jm << (log2m - log2ns - log2r);
                const float2 a0 = base[j];
                const float2 a1 = cmulf(base[j + per_seq], tw[tstep]);
                if (log2r == 2) {
                    const float2 a2 = cmulf(base[j + 2 * per_seq], tw[2 * tstep]);
                    const float2 a3 = cmulf(base[j + 3 * per_seq], tw[3 * tstep]);
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
                dst[c] = seq * stride + ((j - jm) << log2r) + jm;
            }
        }
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int c = 0; c < kWaveBfly; ++c) {
            const int b = lane + c * 64;
            if (b < nbf) {
                buf[dst[c]] = v[c][0];
                buf[dst[c] + ns] = v[c][1];
                if (log2r == 2) {
                    buf[dst[c] + 2 * ns] = v[c][2];
                    buf[dst[c] + 3 * ns] = v[c][3];
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();
        ns <<= log2r;
        log2ns += log2r;
        remaining -= log2r;
    }
}

// Pass 1 unit: range sub-transform p of chirps [m0, m0 + nch) of receiver q.
// Map rows are `row_bytes` apart (N_d times the storage size); the spectra are
// parked as complex64 in the first Mc * 8 bytes of each row.
__device__ __forceinline__ void range_unit(const Geom& g, int nch, size_t row_bytes, const float2* __restrict__ y,
                           char* __restrict__ maps, int m0, int p, int q, float2* lds) {
    const int ms = g.ms, stride = ms + 1;
    float2* buf = lds;                        // [nch][ms + 1]
    float2* pre = buf + nch * stride;         // [ms]
    float2* tw = pre + ms;                    // [ms]
    float2* cen = tw + ms;                    // [ms]
    // the inputs are loaded first so that the table build hides their latency
    const float2* yq = y + ((size_t)q * g.mc + m0) * ms;
    float2 x[kBuf / kThreads];
#pragma unroll
    for (int j = 0; j < kBuf / kThreads; ++j) {
        const int e = threadIdx.x + j * kThreads;
        if (e < nch * ms) x[j] = yq[e];
    }
    fill_tables(pre, tw, cen, p, ms, g.nr, g.centered, false, 1);
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kBuf / kThreads; ++j) {
        const int e = threadIdx.x + j * kThreads;
        if (e < nch * ms) {
            const int c = e >> g.log2_ms, s = e & (ms - 1);
            buf[c * stride + s] = cmulf(x[j], pre[s]);
        }
    }
    __syncthreads();
    lds_fft(buf, nch, stride, g.log2_ms, tw);
    // out bin i = P k + p of chirp m0 + c: Z[q][i][m0 + c], chirps fastest
    const int log2n = 31 - __clz(nch);
    for (int e = threadIdx.x; e < nch * ms; e += kThreads) {
        const int c = e & (nch - 1), k = e >> log2n;
        const float2 v = cmulf(buf[c * stride + k], cen[k]);
        float2* row = reinterpret_cast<float2*>(maps + ((size_t)q * g.nr + (size_t)k * g.pr + p) * row_bytes);
        row[m0 + c] = v;
    }
}

__global__ __launch_bounds__(kThreads) void range_pass(Geom g, int nch, size_t row_bytes, const float2* __restrict__ y,
                                                      char* __restrict__ maps) {
    extern __shared__ float2 lds[];
    range_unit(g, nch, row_bytes, y, maps, blockIdx.x * nch, blockIdx.y, blockIdx.z, lds);
}

// Pass 2 unit: Doppler transforms of range rows [i0, i0 + nrow) of receiver q,
// in place, and the conversion to the storage type DT (half formats: times
// 1 / (Ms Mc)).  With `pre_lds` false (the largest maps) the pre-twiddles are
// evaluated inline instead of from an LDS table.
template <int DT>
__device__ __forceinline__ void doppler_unit(const Geom& g, int nrow, int pre_lds, char* __restrict__ maps, int i0, int q,
                             float2* lds) {
    const int mc = g.mc, pd = g.pd, nd = g.nd, stride = mc + 1;
    const int log2pd = __ffs(pd) - 1;
    float2* buf = lds;                        // [nrow][pd][mc + 1]
    float2* tw = buf + nrow * pd * stride;    // [mc]
    float2* cen = tw + mc;                    // [mc]
    float2* pre = cen + mc;                   // [pd][mc] (pre_lds)
    constexpr int kEs = map_elem_bytes(DT);
    const size_t row_bytes = (size_t)nd * kEs;
    char* rowb = maps + ((size_t)q * g.nr + i0) * row_bytes;
    // the inputs (nrow * mc <= kBuf) are loaded first so that the table build hides their latency
    float2 x[kBuf / kThreads];
#pragma unroll
    for (int j = 0; j < kBuf / kThreads; ++j) {
        const int e = threadIdx.x + j * kThreads;
        if (e < nrow * mc) x[j] = reinterpret_cast<const float2*>(rowb + (size_t)(e >> g.log2_mc) * row_bytes)[e & (mc - 1)];
    }
    fill_tables(pre, tw, cen, 0, mc, nd, g.centered, pre_lds != 0, pre_lds ? pd : 0);
    __syncthreads();
    const int c2 = g.centered ? mc - 1 : 0;
#pragma unroll
    for (int j = 0; j < kBuf / kThreads; ++j) {
        const int e = threadIdx.x + j * kThreads;
        if (e < nrow * mc) {
            const int r = e >> g.log2_mc, m = e & (mc - 1);
            for (int p = 0; p < pd; ++p) {
                const float2 w = pre_lds ? pre[p * mc + m] : expm_pi((long long)p * (2LL * m - c2), nd);
                buf[(r * pd + p) * stride + m] = cmulf(x[j], w);
            }
        }
    }
    __syncthreads();
    lds_fft(buf, nrow * pd, stride, g.log2_mc, tw);
    // out bin l = P k + p, bins fastest
    const float inv_scale = 1.f / map_scale(g.ms, mc, DT);
    for (int e = threadIdx.x; e < nrow * nd; e += kThreads) {
        const int r = e >> g.log2_nd, l = e & (nd - 1);
        const int k = l >> log2pd, p = l & (pd - 1);
        const float2 v = cmulf(buf[(r * pd + p) * stride + k], cen[k]);
        char* row = rowb + (size_t)r * row_bytes;
        if constexpr (DT == GH_MAP_C64) {
            reinterpret_cast<float2*>(row)[l] = v;
        } else {
            reinterpret_cast<uint32_t*>(row)[l] =
                float_to_half_bits(v.x * inv_scale, DT) | (float_to_half_bits(v.y * inv_scale, DT) << 16);
        }
    }
}

// `clear`, when not null, is a caller's counter that the first workgroup sets
// to zero (the Block-OMP selection's split maximum, which runs after the maps).
template <int DT>
__global__ __launch_bounds__(kThreads) void doppler_pass(Geom g, int nrow, int pre_lds, char* __restrict__ maps,
                                                         unsigned* __restrict__ clear) {
    extern __shared__ float2 lds[];
    if (clear && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *clear = 0u;
    doppler_unit<DT>(g, nrow, pre_lds, maps, blockIdx.x * nrow, blockIdx.y, lds);
}

// ---- single frames, one transform set per wave ------------------------------
// Range pass: a workgroup of W waves owns chirps m0 .. m0 + W - 1 of
// sub-transform p of receiver q, one chirp per wave; the workgroup barriers
// are the table build's and the one before the parked store (chirps fastest,
// W consecutive chirps per store run).
template <int NP>
__global__ __launch_bounds__(kThreads) void range_pass_w(Geom g, size_t row_bytes, const float2* __restrict__ y,
                                                        char* __restrict__ maps) {
    extern __shared__ float2 lds[];
    const int nw = blockDim.x >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int ms = g.ms, stride = ms + 1;
    const int m0 = blockIdx.x * nw, p = blockIdx.y, q = blockIdx.z;
    float2* buf = lds;                        // [nw][ms + 1]
    float2* pre = buf + nw * stride;          // [ms]
    float2* tw = pre + ms;                    // [ms]
    float2* cen = tw + ms;                    // [ms]
    const float2* yq = y + ((size_t)q * g.mc + m0 + w) * ms;
    float2 x[NP / 64];
#pragma unroll
    for (int j = 0; j < NP / 64; ++j) {
        const int s = lane + 64 * j;
        if (s < ms) x[j] = yq[s];
    }
    fill_tables(pre, tw, cen, p, ms, g.nr, g.centered, false, 1);
    __syncthreads();
    float2* bw = buf + w * stride;
#pragma unroll
    for (int j = 0; j < NP / 64; ++j) {
        const int s = lane + 64 * j;
        if (s < ms) bw[s] = cmulf(x[j], pre[s]);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    wave_fft<NP>(bw, 1, stride, g.log2_ms, tw);
    __syncthreads();
    // out bin i = P k + p of chirp m0 + c: Z[q][i][m0 + c], chirps fastest
    const int log2n = 31 - __clz(nw);
    for (int e = threadIdx.x; e < nw * ms; e += blockDim.x) {
        const int c = e & (nw - 1), k = e >> log2n;
        const float2 v = cmulf(buf[c * stride + k], cen[k]);
        float2* row = reinterpret_cast<float2*>(maps + ((size_t)q * g.nr + (size_t)k * g.pr + p) * row_bytes);
        row[m0 + c] = v;
    }
}

// Doppler pass: a workgroup of W waves owns range rows i0 .. i0 + W / S - 1
// of receiver q, S waves per row, each with P / S of the row's P
// sub-transforms (S = 1 or 2).  S = 1: the only workgroup barrier is the
// table build's, and each wave overwrites its own row.  S = 2: the two waves
// of a row meet at a second workgroup barrier, after which each writes half
// of the row's bins (the barrier also orders both waves' reads of the parked
// spectra before either overwrites them).  Splitting halves each wave's chain
// of FFT stages and doubles the resident waves.
template <int DT, int NP, int S>
__global__ __launch_bounds__(kThreads) void doppler_pass_w(Geom g, char* __restrict__ maps,
                                                          unsigned* __restrict__ clear) {
    extern __shared__ float2 lds[];
    if (clear && blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) *clear = 0u;
    const int nw = blockDim.x >> 6, w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int mc = g.mc, pd = g.pd, nd = g.nd, stride = mc + 1;
    const int log2pd = __ffs(pd) - 1;
    const int wr = w / S, half = w - wr * S;  // the wave's row in the workgroup, and its part
    const int q = blockIdx.y, row_i = blockIdx.x * (nw / S) + wr;
    const int np = pd / S, p0 = half * np;   // the wave's sub-transforms
    float2* buf = lds;                        // [nw / S][pd][mc + 1]
    float2* tw = buf + (nw / S) * pd * stride;   // [mc]
    float2* cen = tw + mc;                    // [mc]
    float2* pre = cen + mc;                   // [pd][mc]
    constexpr int kEs = map_elem_bytes(DT);
    const size_t row_bytes = (size_t)nd * kEs;
    char* row = maps + ((size_t)q * g.nr + row_i) * row_bytes;
    float2 x[NP / 64];
#pragma unroll
    for (int j = 0; j < NP / 64; ++j) {
        const int m = lane + 64 * j;
        if (m < mc) x[j] = reinterpret_cast<const float2*>(row)[m];
    }
    fill_tables(pre, tw, cen, 0, mc, nd, g.centered, true, pd);
    __syncthreads();
    float2* bw = buf + wr * pd * stride;
#pragma unroll
    for (int j = 0; j < NP / 64; ++j) {
        const int m = lane + 64 * j;
        if (m < mc)
            for (int p = p0; p < p0 + np; ++p) bw[p * stride + m] = cmulf(x[j], pre[p * mc + m]);
    }
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    wave_fft<NP>(bw + p0 * stride, np, stride, g.log2_mc, tw);
    if constexpr (S > 1) __syncthreads();
    // out bin l = P k + p, bins fastest; part `half` writes bins [half nd / S, (half + 1) nd / S)
    const float inv_scale = 1.f / map_scale(g.ms, mc, DT);
    const int l_end = (half + 1) * (nd / S);
    for (int l = half * (nd / S) + lane; l < l_end; l += 64) {
        const int k = l >> log2pd, p = l & (pd - 1);
        const float2 v = cmulf(bw[p * stride + k], cen[k]);
        if constexpr (DT == GH_MAP_C64) {
            reinterpret_cast<float2*>(row)[l] = v;
        } else {
            reinterpret_cast<uint32_t*>(row)[l] =
                float_to_half_bits(v.x * inv_scale, DT) | (float_to_half_bits(v.y * inv_scale, DT) << 16);
        }
    }
}

// Waves per workgroup of the one-transform-per-wave passes (a power of two
// from 8 down to 2 that fits 64 KB of LDS and divides the chirps or rows), or
// 0 when a wave's transforms exceed kWavePts or the LDS.
int range_waves(const Geom& g) {
    if (g.ms > kWavePts) return 0;
    for (int w = 8; w >= 2; w >>= 1) {
        const size_t lds = ((size_t)w * (g.ms + 1) + 3 * (size_t)g.ms) * sizeof(float2);
        if (lds <= 65536 && g.mc % w == 0) return w;
    }
    return 0;
}

// Doppler: waves per row S = 2 when the row has an even number of
// sub-transforms, else 1; W / S rows per workgroup.
int doppler_split(const Geom& g) { return g.pd >= 2 ? 2 : 1; }

size_t doppler_w_lds(const Geom& g, int w) {
    return ((size_t)(w / doppler_split(g)) * g.pd * (g.mc + 1) + (2 + (size_t)g.pd) * g.mc) * sizeof(float2);
}

int doppler_waves(const Geom& g) {
    const int sp = doppler_split(g);
    if ((long)g.pd * g.mc / sp > kWavePts) return 0;
    for (int w = 8; w >= 2; w >>= 1)
        if (doppler_w_lds(g, w) <= 65536 && g.nr % (w / sp) == 0) return w;
    return 0;
}

// ---- batches: persistent launches over the work units of many frames ----------
// A workgroup walks units u = blockIdx.x, blockIdx.x + gridDim.x, ... in
// increasing order, so its frame index only moves forward; it keeps the
// current frame's descriptor in LDS and reloads it when the frame changes.

// Advance f to the frame holding unit u (all threads agree; unit u exists).
__device__ __forceinline__ int advance_frame(const FrameDesc* __restrict__ frames, int nf, int f, int u, int which) {
    while (f + 1 < nf && frames[f + 1].unit0[which] <= u) ++f;
    return f;
}

// Copy one frame descriptor into LDS (all threads; bracketed by barriers).
__device__ __forceinline__ void load_frame(const FrameDesc* src, FrameDesc* dst) {
    static_assert(sizeof(FrameDesc) % 4 == 0, "descriptor copied as 32-bit words");
    __syncthreads();
    const int* s = reinterpret_cast<const int*>(src);
    int* d = reinterpret_cast<int*>(dst);
    for (int i = threadIdx.x; i < (int)(sizeof(FrameDesc) / 4); i += blockDim.x) d[i] = s[i];
    __syncthreads();
}

__global__ __launch_bounds__(kThreads) void range_batch(const FrameDesc* __restrict__ frames, int nf, int total) {
    extern __shared__ float2 lds[];
    __shared__ FrameDesc fd;
    int f = 0, loaded = -1;
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        f = advance_frame(frames, nf, f, u, 0);
        if (f != loaded) {
            load_frame(frames + f, &fd);
            loaded = f;
        }
        const int lu = u - fd.unit0[0];
        if (lu >= fd.nunit[0]) continue;   // not reached for a consistent table
        const int groups = fd.g.mc / fd.nch;
        const int q = lu / (fd.g.pr * groups), rem = lu - q * fd.g.pr * groups;
        const int p = rem / groups, grp = rem - p * groups;
        range_unit(fd.g, fd.nch, (size_t)fd.g.nd * 8, as_global(fd.y), as_global(fd.maps), grp * fd.nch, p, q, lds);
        __syncthreads();   // the next unit reuses the LDS buffers
    }
}

__global__ __launch_bounds__(kThreads) void doppler_batch(const FrameDesc* __restrict__ frames, int nf, int total) {
    extern __shared__ float2 lds[];
    __shared__ FrameDesc fd;
    int f = 0, loaded = -1;
    for (int u = blockIdx.x; u < total; u += gridDim.x) {
        f = advance_frame(frames, nf, f, u, 1);
        if (f != loaded) {
            load_frame(frames + f, &fd);
            loaded = f;
        }
        const int lu = u - fd.unit0[1];
        if (lu >= fd.nunit[1]) continue;
        const int groups = fd.g.nr / fd.nrow;
        const int q = lu / groups, grp = lu - q * groups;
        doppler_unit<GH_MAP_C64>(fd.g, fd.nrow, fd.pre_lds, as_global(fd.maps), grp * fd.nrow, q, lds);
        __syncthreads();
    }
}

}  // namespace

// Work decomposition of the two passes (shared by single frames and batches).
void rd_maps_plan(const Geom& g, int& nch, size_t& lds1, int& nrow, int& pre_lds, size_t& lds2) {
    // range pass: chirps per workgroup, halved (down to 8) until there are >= 512 workgroups
    nch = kBuf / g.ms;
    if (nch > g.mc) nch = g.mc;
    while (nch > 8 && (long)(g.mc / nch) * g.pr * g.k < 512) nch >>= 1;
    nrow = kBuf / g.nd;
    rd_maps_shape(g, nch, nrow, lds1, pre_lds, lds2);
}

// Clamps nch and nrow (powers of two) to what one workgroup holds (nch Ms and
// nrow N_d at most kBuf values, no more than the frame) and gives the LDS of
// both passes.
void rd_maps_shape(const Geom& g, int& nch, int& nrow, size_t& lds1, int& pre_lds, size_t& lds2) {
    if (nch > kBuf / g.ms) nch = kBuf / g.ms;
    if (nch > g.mc) nch = g.mc;
    if (nch < 1) nch = 1;
    if (nrow > kBuf / g.nd) nrow = kBuf / g.nd;
    if (nrow > g.nr) nrow = g.nr;
    if (nrow < 1) nrow = 1;
    lds1 = ((size_t)nch * (g.ms + 1) + 3 * (size_t)g.ms) * sizeof(float2);
    lds2 = ((size_t)nrow * g.pd * (g.mc + 1) + 2 * (size_t)g.mc) * sizeof(float2);
    pre_lds = lds2 + (size_t)g.nd * sizeof(float2) <= 65536 ? 1 : 0;
    if (pre_lds) lds2 += (size_t)g.nd * sizeof(float2);
}

int range_batch_max_workgroups(size_t lds) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, range_batch, kThreads, lds) != hipSuccess) return 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

int doppler_batch_max_workgroups(size_t lds) {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, doppler_batch, kThreads, lds) != hipSuccess) return 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

hipError_t launch_rd_maps_batch(const FrameDesc* frames, int nf, int range_units, int doppler_units, size_t lds1,
                                size_t lds2, int wg_range, int wg_doppler, hipStream_t st) {
    const int w1 = wg_range < range_units ? wg_range : range_units;
    hipLaunchKernelGGL(range_batch, dim3(w1), dim3(kThreads), lds1, st, frames, nf, range_units);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int w2 = wg_doppler < doppler_units ? wg_doppler : doppler_units;
    hipLaunchKernelGGL(doppler_batch, dim3(w2), dim3(kThreads), lds2, st, frames, nf, doppler_units);
    return hipGetLastError();
}

hipError_t launch_range_spectra(const Geom& g, const float2* y, float2* spectra, hipStream_t st) {
    int nch, nrow, pre_lds;
    size_t lds1, lds2;
    rd_maps_plan(g, nch, lds1, nrow, pre_lds, lds2);
    hipLaunchKernelGGL(range_pass, dim3(g.mc / nch, g.pr, g.k), dim3(kThreads), lds1, st, g, nch,
                       (size_t)g.mc * sizeof(float2), y, reinterpret_cast<char*>(spectra));
    return hipGetLastError();
}

hipError_t launch_rd_maps(const Geom& g, const float2* y, void* maps_v, int map_dtype, hipStream_t st,
                          unsigned* clear) {
    char* maps = static_cast<char*>(maps_v);
    const size_t row_bytes = (size_t)g.nd * map_elem_bytes(map_dtype);
    int nch, nrow, pre_lds;
    size_t lds1, lds2;
    rd_maps_plan(g, nch, lds1, nrow, pre_lds, lds2);
    const int w1 = range_waves(g), w2 = doppler_waves(g);
    if (w1 > 0) {
        const size_t l = ((size_t)w1 * (g.ms + 1) + 3 * (size_t)g.ms) * sizeof(float2);
        const dim3 grid(g.mc / w1, g.pr, g.k), blk(64 * w1);
        if (g.ms <= 256)
            hipLaunchKernelGGL(range_pass_w<256>, grid, blk, l, st, g, row_bytes, y, maps);
        else
            hipLaunchKernelGGL(range_pass_w<512>, grid, blk, l, st, g, row_bytes, y, maps);
    } else {
        hipLaunchKernelGGL(range_pass, dim3(g.mc / nch, g.pr, g.k), dim3(kThreads), lds1, st, g, nch, row_bytes, y,
                           maps);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (w2 > 0) {
        const int sp = doppler_split(g);
        const size_t l = doppler_w_lds(g, w2);
        const dim3 grid(g.nr / (w2 / sp), g.k), blk(64 * w2);
        const int pts = g.pd * g.mc / sp;   // points per wave
#define GH_DOPPLER_W(DT)                                                                            \
    do {                                                                                            \
        if (sp == 1 && pts <= 256)                                                                  \
            hipLaunchKernelGGL((doppler_pass_w<DT, 256, 1>), grid, blk, l, st, g, maps, clear);     \
        else if (sp == 1)                                                                           \
            hipLaunchKernelGGL((doppler_pass_w<DT, 512, 1>), grid, blk, l, st, g, maps, clear);     \
        else if (pts <= 256)                                                                        \
            hipLaunchKernelGGL((doppler_pass_w<DT, 256, 2>), grid, blk, l, st, g, maps, clear);     \
        else                                                                                        \
            hipLaunchKernelGGL((doppler_pass_w<DT, 512, 2>), grid, blk, l, st, g, maps, clear);     \
    } while (0)
        if (map_dtype == GH_MAP_F16)
            GH_DOPPLER_W(GH_MAP_F16);
        else if (map_dtype == GH_MAP_BF16)
            GH_DOPPLER_W(GH_MAP_BF16);
        else
            GH_DOPPLER_W(GH_MAP_C64);
#undef GH_DOPPLER_W
        return hipGetLastError();
    }
    const dim3 grid2(g.nr / nrow, g.k);
    if (map_dtype == GH_MAP_F16)
        hipLaunchKernelGGL(doppler_pass<GH_MAP_F16>, grid2, dim3(kThreads), lds2, st, g, nrow, pre_lds, maps,
                           clear);
    else if (map_dtype == GH_MAP_BF16)
        hipLaunchKernelGGL(doppler_pass<GH_MAP_BF16>, grid2, dim3(kThreads), lds2, st, g, nrow, pre_lds, maps,
                           clear);
    else
        hipLaunchKernelGGL(doppler_pass<GH_MAP_C64>, grid2, dim3(kThreads), lds2, st, g, nrow, pre_lds, maps,
                           clear);
    return hipGetLastError();
}

}  // namespace gh
