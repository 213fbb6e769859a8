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
// Matrix-core mapping of the FP32 range zoom and the generating Doppler zoom
// (64-lane wave, 16 x 16 output tile, FP32 accumulation):
//   lane = r + 16 g holds contraction indices k0 + 8 g + e (e = 0..7) of row r
//   of the left operand and of column r of the right operand.  FP32 issues
//   eight 16x16x4 products, the e-th taking element e of every lane (any
//   assignment of contraction indices to the k slots is valid if both
//   operands share it).  The output element (i, j) sits in lane j + 16 (i / 4),
//   slot i % 4.
// FP32 range zoom: a complex product is four real ones,
//   Re C += Re A Re B - Im A Im B,  Im C += Re A Im B + Im A Re B;
// atoms are generated in registers: one exact anchor per run of eight from a
// 32-bit fixed-point phase (the wrap modulo one cycle is integer overflow),
// then the recurrence e_{n+1} = e_n exp(-j 2 pi f).
// BF16 (gemm_dtype BF16): complex products over interleaved (re, im) pairs,
// two 16x16x32 products per complex tile step; the range zoom stages the frame
// in LDS once per workgroup.
// Both precisions: the range zoom leaves h = G times a chirp, and the Doppler
// zoom reads its left operand from a chirp (Toeplitz) table and forms its
// right one from h and a second chirp table (see the kernels below).  Slabs
// of more than 16 velocity tiles, or tables beyond 64 KB of LDS, take the
// generating Doppler zoom on G instead.
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

// High word of (a * b) mod 2^64 for a 64-bit fixed-point a and a 32-bit integer b.
__device__ __forceinline__ uint32_t fixed_mul_hi(uint64_t a, uint32_t b) {
    return (uint32_t)(a >> 32) * b + __umulhi((uint32_t)a, b);
}

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

// Range zoom (FP32), G_q[x][m] (complex64 [K][Nloc][Mc]).  Grid
// (ceil(Nloc / 64), ceil(Mc / 64), K); wave w of a workgroup owns 16
// locations and 64 chirps of receiver blockIdx.z.
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
            mfma_complex<false>(a, b, cre[t], cim[t]);
        }
    }
    // output element (location 4 seg + e, chirp r) of each tile
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

// Range zoom (FP32) for the chirp-table Doppler zoom:
//   h_q[x][m] = G_q[x][m] exp(-j 2 pi (f0 m + (fx + fy) m^2 / 2))   (complex64 [K][Nloc][Mc]).
// The samples are split over the waves of a workgroup: with nsplit parts
// (4 for Ms >= 128, 2 for Ms = 64, else 1), the workgroup owns 4 / nsplit
// tiles of 16 locations x 64 chirps of receiver blockIdx.z, and wave
// (tile, part) sums samples [part Ms / nsplit, (part + 1) Ms / nsplit).  The
// partial sums meet in LDS and are added in part order; the wave of part p
// finishes the chirp tiles p, p + nsplit, ... (chirp factor and store).
// Grid (ceil(Nloc / (64 / nsplit)), ceil(Mc / 64), K).  Four times the waves
// of the unsplit kernel at equal work: it shares the device better with the
// refinement that runs beside it in a step.
__global__ __launch_bounds__(kThreads) void direct_range_zoom_chirp(Geom g, GridP gp, const float2* __restrict__ y,
                                                                   float2* __restrict__ hws, int nsplit) {
    __shared__ f32x4 part[kWaves][2 * kNT][64];
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int seg = lane >> 4;
    const int w = threadIdx.x >> 6;
    const int lg = w / nsplit, sp = w - lg * nsplit;   // location tile in the workgroup, sample part
    const int q = blockIdx.z;
    const int loc0 = (blockIdx.x * (kWaves / nsplit) + lg) * 16;
    const int m0 = blockIdx.y * (16 * kNT);
    const int ms = g.ms, mc = g.mc;
    const int s_begin = sp * (ms / nsplit), s_end = s_begin + ms / nsplit;

    uint32_t fr = 0;
    uint64_t f0l = 0, hsl = 0;
    if (loc0 + r < gp.nloc) {
        const int loc = loc0 + r;
        const int ix = loc / gp.n[1], iy = loc - ix * gp.n[1];
        double rr, wx, wy;
        bistatic(g, q, gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], rr, wx, wy);
        fr = cycles_to_fixed(g.fr_per_m * rr);
        f0l = cycles_to_fixed64(g.fd_per_mps * (wx * gp.lo[2] + wy * gp.lo[3]));
        hsl = cycles_to_fixed64(0.5 * g.fd_per_mps * (wx * gp.step[2] + wy * gp.step[3]));
    }
    const float2 ratio = expm_fixed(fr);

    f32x4 cre[kNT], cim[kNT];
#pragma unroll
    for (int t = 0; t < kNT; ++t) cre[t] = cim[t] = zero4();

    const float2* yq = y + (size_t)q * mc * ms;
    for (int s0 = s_begin; s0 < s_end; s0 += 32) {
        const int sb = s0 + seg * kRun;
        const bool live = sb < s_end;   // a part is a multiple of 32 samples, or all of Ms (a power of two >= 8)
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
            mfma_complex<false>(a, b, cre[t], cim[t]);
        }
    }
    // output element (location 4 seg + e, chirp r) of each tile; the chirp
    // rates of location 4 seg + e come from lane 4 seg + e
    uint64_t f0e[4], hse[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int src = 4 * seg + e;
        f0e[e] = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(f0l >> 32), src, 64) << 32) |
                 (uint32_t)__shfl((int)(uint32_t)f0l, src, 64);
        hse[e] = ((uint64_t)(uint32_t)__shfl((int)(uint32_t)(hsl >> 32), src, 64) << 32) |
                 (uint32_t)__shfl((int)(uint32_t)hsl, src, 64);
    }
#pragma unroll
    for (int t = 0; t < kNT; ++t) {
        part[w][2 * t][lane] = cre[t];
        part[w][2 * t + 1][lane] = cim[t];
    }
    __syncthreads();
    const int w0 = lg * nsplit;
    for (int t = sp; t < kNT; t += nsplit) {
        f32x4 sr = part[w0][2 * t][lane], si = part[w0][2 * t + 1][lane];
        for (int p = 1; p < nsplit; ++p) {
            sr += part[w0 + p][2 * t][lane];
            si += part[w0 + p][2 * t + 1][lane];
        }
        const int m = m0 + t * 16 + r;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int loc = loc0 + 4 * seg + e;
            if (loc < gp.nloc && m < mc) {
                const uint32_t ph = fixed_mul_hi(f0e[e], (uint32_t)m) + fixed_mul_hi(hse[e], (uint32_t)(m * m));
                hws[((size_t)q * gp.nloc + loc) * mc + m] = cmul(make_float2(sr[e], si[e]), expm_fixed(ph));
            }
        }
    }
}

// ---- BF16 operands ----------------------------------------------------------
// A complex product as real ones over interleaved (re, im) pairs: contraction
// slot 2k + c of a 16x16x32 BF16 product holds the real (c = 0) or imaginary
// (c = 1) part of complex index k, so one product contracts 16 complex
// indices.  With the right operand b laid out (br, bi) per index and the left
// one in the two forms (ar, -ai) and (ai, ar),
//   Re(a b) = ar br - ai bi   and   Im(a b) = ai br + ar bi
// take two products instead of four.  Lane r + 16 g holds complex indices
// 4 g .. 4 g + 3 of row r (left operand) or column r (right operand).

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float fvec2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t bf16_pair(float lo, float hi) {
    return __builtin_bit_cast(uint32_t, __builtin_convertvector((fvec2){lo, hi}, bf16x2));
}
__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }
__device__ __forceinline__ bf16x2 as_bf16x2(uint32_t v) { return __builtin_bit_cast(bf16x2, v); }

// BF16 dot product of two (x, y) pairs with an FP32 result, a.x b.x + a.y b.y
__device__ __forceinline__ float dot2_bf16(uint32_t a, uint32_t b) {
    return __builtin_amdgcn_fdot2_f32_bf16(as_bf16x2(a), as_bf16x2(b), 0.f, false);
}

struct ToepPlan {
    int ex, ey, mcp, words;   // table lengths and 32-bit words per receiver
};

__host__ __device__ inline ToepPlan toep_plan(int mc, int nvx, int nvy) {
    ToepPlan p;
    p.mcp = mc < 16 ? 16 : mc;
    p.ex = (p.mcp + ((nvx + 15) & ~15) - 1 + 3) & ~3;
    p.ey = (p.mcp + ((nvy + 15) & ~15) - 1 + 3) & ~3;
    p.words = 2 * p.ex + 2 * p.ey + p.mcp;
    return p;
}

// exp(-j 2 pi ph 2^-32) in FP32: the nearest quarter turn from the top bits,
// the remainder (at most an eighth of a turn, converted from a 30-bit integer)
// through the Taylor series of sine (to x^9) and cosine (to x^10); truncation
// below 2e-9 on [-pi/4, pi/4], measured maximum error 1.2e-7 over all phases.
__device__ __forceinline__ float2 expm_poly(uint32_t ph) {
    const uint32_t qn = (ph + 0x20000000u) >> 30;
    const int32_t d = (int32_t)(ph - (qn << 30));
    const float x = (float)d * 1.4629180792671596e-09f;   // 2 pi / 2^32
    const float x2 = x * x;
    float ps = fmaf(x2, 2.7557319e-06f, -1.9841270e-04f);   // 1/9!, -1/7!
    ps = fmaf(x2, ps, 8.3333333e-03f);                       // 1/5!
    ps = fmaf(x2, ps, -1.6666667e-01f);                      // -1/3!
    const float sn = fmaf(x * x2, ps, x);
    float pc = fmaf(x2, -2.7557319e-07f, 2.4801587e-05f);   // -1/10!, 1/8!
    pc = fmaf(x2, pc, -1.3888889e-03f);                      // -1/6!
    pc = fmaf(x2, pc, 4.1666667e-02f);                       // 1/4!
    pc = fmaf(x2, pc, -0.5f);
    const float cs = fmaf(x2, pc, 1.0f);
    // rotate by qn quarter turns: (cos, sin) of qn pi/2 + x
    const bool odd = qn & 1, neg_c = (qn + 1) & 2, neg_s = qn & 2;
    float co = odd ? sn : cs, si = odd ? cs : sn;
    co = neg_c ? -co : co;
    si = neg_s ? -si : si;
    return make_float2(co, -si);
}

// exp(-j 2 pi ph 2^-32) from the hardware sine and cosine (argument in revolutions)
__device__ __forceinline__ float2 expm_hw(uint32_t ph) {
    const float x = __uint2float_rn(ph) * 2.3283064365386963e-10f;   // 2^-32
    return make_float2(__builtin_amdgcn_cosf(x), -__builtin_amdgcn_sinf(x));
}



// Range zoom with BF16 operands.  A workgroup owns 64 LT locations x 16 CT
// chirps of one receiver; wave w owns locations 16 LT w .. 16 LT (w + 1) - 1.
// The frame's chirps are staged in LDS as BF16 pairs, 64 samples at a time
// (double-buffered; rows padded by 16 bytes so the operand reads of 16 rows
// fall in distinct banks), once for the four waves.  Each lane keeps the
// atoms of its locations at its four sample slots in FP32 and advances them
// by exp(-j 2 pi 16 f_r) per 16-sample step, rounding to BF16 only as
// operands.
//   CHIRP = false: G_q[x][m] (complex64 [K][Nloc][Mc]), as the FP32 path.
//   CHIRP = true:  h_q[x][m] = G_q[x][m] exp(-j 2 pi (f0 m + (fx + fy) m^2 / 2))
//                  as BF16 pairs ([K][Nloc][mcp] 32-bit words, mcp = max(Mc, 16);
//                  words m >= Mc are not written), the right-hand factor of
//                  the chirp-table Doppler zoom below.
constexpr int kRzChunk = 64;                 // samples per staged chunk
constexpr int kRzRowWords = kRzChunk + 4;    // BF16 pairs per staged row (+16 bytes)

template <int LT, int CT, bool CHIRP>
__global__ __launch_bounds__(kThreads) void direct_range_zoom_bf16(Geom g, GridP gp, const float2* __restrict__ y,
                                                                  void* __restrict__ out) {
    constexpr int kRows = 16 * CT;                 // chirps per workgroup
    constexpr int kTpr = kThreads / kRows;         // staging threads per row
    constexpr int kSpt = kRzChunk / kTpr;          // samples per staging thread (4 CT)
    __shared__ __attribute__((aligned(16))) uint32_t ys[2][kRows * kRzRowWords];
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int seg = lane >> 4;
    const int q = blockIdx.z;
    const int loc0 = (blockIdx.x * kWaves + (threadIdx.x >> 6)) * 16 * LT;
    const int m0 = blockIdx.y * kRows;
    const int ms = g.ms, mc = g.mc;
    const int chunk = ms < kRzChunk ? ms : kRzChunk;
    const int ksteps = (chunk + 15) >> 4;

    // location 16 lt + r: atoms at samples 4 seg .. 4 seg + 3, the 16-sample step
    // factor, and (CHIRP) the Doppler chirp rates in 64-bit fixed point
    float2 at[LT][4], rho[LT];
    uint64_t f0l[LT], hsl[LT];
#pragma unroll
    for (int lt = 0; lt < LT; ++lt) {
        uint32_t fr = 0;
        f0l[lt] = hsl[lt] = 0;
        const int loc = loc0 + 16 * lt + r;
        if (loc < gp.nloc) {
            const int ix = loc / gp.n[1], iy = loc - ix * gp.n[1];
            double rr, wx, wy;
            bistatic(g, q, gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], rr, wx, wy);
            fr = cycles_to_fixed(g.fr_per_m * rr);
            if constexpr (CHIRP) {
                f0l[lt] = cycles_to_fixed64(g.fd_per_mps * (wx * gp.lo[2] + wy * gp.lo[3]));
                hsl[lt] = cycles_to_fixed64(0.5 * g.fd_per_mps * (wx * gp.step[2] + wy * gp.step[3]));
            }
        }
        const float2 r1 = expm_fixed(fr);
        at[lt][0] = expm_fixed(fr * (uint32_t)(4 * seg));
#pragma unroll
        for (int e = 1; e < 4; ++e) at[lt][e] = cmul(at[lt][e - 1], r1);
        rho[lt] = expm_fixed(fr * 16u);
    }

    f32x4 cre[LT][CT], cim[LT][CT];
#pragma unroll
    for (int lt = 0; lt < LT; ++lt)
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) cre[lt][ct] = cim[lt][ct] = zero4();

    // staging: thread t -> chirp m0 + t / kTpr, samples kSpt (t % kTpr) .. + kSpt - 1 of the chunk
    const int srow = threadIdx.x / kTpr, spart = threadIdx.x % kTpr;
    const bool row_ok = m0 + srow < mc;
    const float4* ysrc = reinterpret_cast<const float4*>(y + ((size_t)q * mc + (row_ok ? m0 + srow : 0)) * ms);
    float4 st[kSpt / 2];
    auto load_chunk = [&](int s0) {
#pragma unroll
        for (int i = 0; i < kSpt / 2; ++i) {
            const int s = s0 + kSpt * spart + 2 * i;
            st[i] = (row_ok && s < ms) ? ysrc[s >> 1] : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    auto store_chunk = [&](int b) {
        u32x4* dst = reinterpret_cast<u32x4*>(ys[b] + srow * kRzRowWords + kSpt * spart);
#pragma unroll
        for (int i = 0; i < kSpt / 4; ++i)
            dst[i] = u32x4{bf16_pair(st[2 * i].x, st[2 * i].y), bf16_pair(st[2 * i].z, st[2 * i].w),
                           bf16_pair(st[2 * i + 1].x, st[2 * i + 1].y), bf16_pair(st[2 * i + 1].z, st[2 * i + 1].w)};
    };

    load_chunk(0);
    store_chunk(0);
    __syncthreads();
    int buf = 0;
    for (int s0 = 0; s0 < ms; s0 += chunk) {
        const bool more = s0 + chunk < ms;
        if (more) load_chunk(s0 + chunk);
        for (int k = 0; k < ksteps; ++k) {
            u32x4 b[CT];
#pragma unroll
            for (int ct = 0; ct < CT; ++ct)
                b[ct] = *reinterpret_cast<const u32x4*>(ys[buf] + (16 * ct + r) * kRzRowWords + 16 * k + 4 * seg);
#pragma unroll
            for (int lt = 0; lt < LT; ++lt) {
                u32x4 are, aim;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    are[e] = bf16_pair(at[lt][e].x, -at[lt][e].y);
                    aim[e] = bf16_pair(at[lt][e].y, at[lt][e].x);
                    at[lt][e] = cmul(at[lt][e], rho[lt]);
                }
#pragma unroll
                for (int ct = 0; ct < CT; ++ct) {
                    cre[lt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(are), as_bf16x8(b[ct]),
                                                                          cre[lt][ct], 0, 0, 0);
                    cim[lt][ct] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(aim), as_bf16x8(b[ct]),
                                                                          cim[lt][ct], 0, 0, 0);
                }
            }
        }
        if (more) store_chunk(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    // output element (location 4 seg + e, chirp r) of each tile.  The chirp's
    // phase is taken in 32-bit fixed point (the rates' top 32 bits): at most
    // (Mc + Mc^2) 2^-32 cycles off (4e-6 at Mc = 128, 1.5e-5 at Mc = 256),
    // far below the 2^-8 relative rounding of the BF16 result.
#pragma unroll
    for (int lt = 0; lt < LT; ++lt) {
        uint32_t f0e[4], hse[4];
        if constexpr (CHIRP) {
#pragma unroll
            for (int e = 0; e < 4; ++e) {   // rates of location 4 seg + e, computed by lane 4 seg + e
                const int src = 4 * seg + e;
                f0e[e] = (uint32_t)__shfl((int)(uint32_t)(f0l[lt] >> 32), src, 64);
                hse[e] = (uint32_t)__shfl((int)(uint32_t)(hsl[lt] >> 32), src, 64);
            }
        }
#pragma unroll
        for (int ct = 0; ct < CT; ++ct) {
            const int m = m0 + 16 * ct + r;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int loc = loc0 + 16 * lt + 4 * seg + e;
                if (loc < gp.nloc && m < mc) {
                    if constexpr (CHIRP) {
                        const int mcp = mc < 16 ? 16 : mc;
                        const uint32_t ph = f0e[e] * (uint32_t)m + hse[e] * (uint32_t)(m * m);
                        const float2 hv = cmul(make_float2(cre[lt][ct][e], cim[lt][ct][e]), expm_hw(ph));
                        static_cast<uint32_t*>(out)[((size_t)q * gp.nloc + loc) * mcp + m] = bf16_pair(hv.x, hv.y);
                    } else {
                        static_cast<float2*>(out)[((size_t)q * gp.nloc + loc) * mc + m] =
                            make_float2(cre[lt][ct][e], cim[lt][ct][e]);
                    }
                }
            }
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

// Slab epilogue of the chirp-table Doppler zooms: tile t of the velocity slab
// (row tile t % tiles_x, column tile t / tiles_x) holds output (16 tx + 4 g + e,
// 16 ty + r) in lane r + 16 g, slot e.  Writes the slab (if dec) and the block
// maximum of location loc (ties to the lowest index, excluded cells skipped).
template <int MAXT>
__device__ __forceinline__ void slab_peak(const f32x4 (&dsum)[MAXT], int ntiles, int tiles_x, int nvx, int nvy,
                                          int64_t base, int lane, float* __restrict__ dec,
                                          gh_peak* __restrict__ block, int loc, const int64_t* __restrict__ excl,
                                          int nexcl) {
    const int r = lane & 15, seg = lane >> 4;
    float best_v = -INFINITY;
    int best_i = 0x7fffffff;
#pragma unroll
    for (int t = 0; t < MAXT; ++t) {
        if (t < ntiles) {
            const int ty = t / tiles_x, tx = t - ty * tiles_x;
            const int ivy = ty * 16 + r;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int ivx = tx * 16 + 4 * seg + e;
                if (ivx < nvx && ivy < nvy) {
                    const int v = ivx * nvy + ivy;
                    if (dec) dec[base + v] = dsum[t][e];
                    bool skip = false;
                    for (int i = 0; i < nexcl; ++i) skip |= (excl[i] == base + v);
                    if (!skip) peak_merge(best_v, best_i, dsum[t][e], v);
                }
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

// Doppler zoom with BF16 operands through chirp tables.  With
// f_d = f0 + ivx fx + ivy fy and 2 ivx m = ivx^2 + m^2 - (ivx - m)^2 (likewise
// for ivy), the correlation of one receiver is
//   c[ivx][ivy] = exp(-j pi (fx ivx^2 + fy ivy^2)) sum_m h[m] Tx[ivx - m] Ty[ivy - m],
//   h[m] = G[m] exp(-j 2 pi (f0 m + (fx + fy) m^2 / 2)),
//   Tx[k] = exp(j pi fx k^2),  Ty[k] = exp(j pi fy k^2);
// the leading factor has modulus one and drops out of |c|^2.  The left operand
// (rows ivx, contraction m) is the Toeplitz matrix Tx[ivx - m], read from a
// table of Mc + 15 values per 16-row tile span; the right one is h[m] Ty[ivy - m],
// formed per element by two BF16 dot products (its real and imaginary parts).
// A (location, receiver) pair thus generates O(Mc + Nvx + Nvy) values instead
// of O(Mc (Nvx + Nvy)).
//
// One wave per location, receivers in turn.  For receiver q the wave writes,
// into its own LDS region, the chirp tables in both left-operand forms
// (tx1 = (re, -im), tx2 = (im, re) of Tx; ty1, ty2 likewise of Ty) and h as
// BF16 pairs:
//   tx[n], n in [0, ex):  Tx[k] with k = nvx_pad - 1 - n (so a lane's four
//                         contraction slots read four consecutive entries)
//   ty[n], n in [0, ey):  Ty[k] with k = nvy_pad - 1 - n
//   h[m],  m in [0, mcp): zero for m >= Mc
// then walks the 16 x 16 tiles of the velocity slab column tile by column
// tile: the right-operand fragments h[m] Ty[ivy - m] of a column tile are
// formed once, in registers, for all its row tiles.  |c_q|^2 accumulates per
// tile in registers across receivers (at most MAXT tiles).  STEPS > 0 is the
// exact number of 16-chirp steps, mcp / 16 (the right operands cached, the
// loops unrolled without guards); STEPS = 0 forms the right operand step by
// step (Mc > 128).  h of the next receiver is loaded while the current one is
// in work.
// Phases are 64-bit fixed point in cycles; the table values come from the
// hardware sine and cosine (absolute error near 1e-6, far below the BF16
// rounding of the operands they feed).
template <int MAXT, int STEPS>
__global__ __launch_bounds__(kThreads) void direct_doppler_zoom_chirp(Geom g, GridP gp, ToepPlan tp,
                                                                     const uint32_t* __restrict__ hws,
                                                                     float* __restrict__ dec,
                                                                     gh_peak* __restrict__ block,
                                                                     const int64_t* __restrict__ excl, int nexcl) {
    constexpr bool STREAM = STEPS == 0;
    constexpr int MAXS = STREAM ? 1 : STEPS;
    extern __shared__ __attribute__((aligned(16))) uint32_t toep_lds[];
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int seg = lane >> 4;
    const int w = threadIdx.x >> 6;
    const int loc = blockIdx.x * (blockDim.x >> 6) + w;
    if (loc >= gp.nloc) return;   // wave-uniform; the kernel has no workgroup barrier
    uint32_t* tx1 = toep_lds + (size_t)w * tp.words;
    uint32_t* tx2 = tx1 + tp.ex;
    uint32_t* ty1 = tx2 + tp.ex;
    uint32_t* ty2 = ty1 + tp.ey;
    uint32_t* hh = ty2 + tp.ey;
    const int ix = loc / gp.n[1], iy = loc - ix * gp.n[1];
    const int nvx = gp.n[2], nvy = gp.n[3], nv = gp.nv, mc = g.mc;
    const int nvxp = (nvx + 15) & ~15, nvyp = (nvy + 15) & ~15;
    const int tiles_x = nvxp >> 4, ntiles = tiles_x * (nvyp >> 4);
    const int kx = (nvxp > tp.mcp ? nvxp : tp.mcp) - 1, ky = (nvyp > tp.mcp ? nvyp : tp.mcp) - 1;
    const int steps = STREAM ? tp.mcp >> 4 : STEPS;

    constexpr int kHw = (16 * MAXS + 63) / 64;   // h words per lane held ahead (cached path)
    uint32_t hpre[kHw];
    auto load_h = [&](int q) {
        const uint32_t* hq = hws + ((size_t)q * gp.nloc + loc) * tp.mcp;
#pragma unroll
        for (int u = 0; u < kHw; ++u) {
            const int m = lane + 64 * u;
            hpre[u] = m < mc ? hq[m] : 0u;
        }
    };
    if (!STREAM) load_h(0);

    // receiver `lane`: fx / 2 and fy / 2 in 64-bit fixed point
    uint64_t hxl = 0, hyl = 0;
    if (lane < g.k) {
        double rr, wx, wy;
        bistatic(g, lane, gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], rr, wx, wy);
        hxl = cycles_to_fixed64(0.5 * g.fd_per_mps * wx * gp.step[2]);
        hyl = cycles_to_fixed64(0.5 * g.fd_per_mps * wy * gp.step[3]);
    }
    auto bcast64 = [](uint64_t v, int src) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
        return ((uint64_t)hi << 32) | lo;
    };

    f32x4 dsum[MAXT];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) dsum[t] = zero4();

    for (int q = 0; q < g.k; ++q) {
        // every lane has finished reading receiver q - 1's tables (in-order LDS per wave)
        __builtin_amdgcn_wave_barrier();
        if constexpr (STREAM) {
            const uint32_t* hq = hws + ((size_t)q * gp.nloc + loc) * tp.mcp;
            for (int m = lane; m < tp.mcp; m += 64) hh[m] = m < mc ? hq[m] : 0u;
        } else {
#pragma unroll
            for (int u = 0; u < kHw; ++u) {
                const int m = lane + 64 * u;
                if (m < tp.mcp) hh[m] = hpre[u];
            }
            if (q + 1 < g.k) load_h(q + 1);
        }
        const uint64_t hx = bcast64(hxl, q), hy = bcast64(hyl, q);
        // the tables are even in k and the tiles read |k| <= max(nv_pad, mcp) - 1:
        // one value per |k|, stored at k and -k.  With Mc <= 32 (at most two steps)
        // and each table at most 32 values, both are made in one pass of the wave:
        // lanes 0-31 Tx, lanes 32-63 Ty.
        bool one_pass = false;
        if constexpr (!STREAM && MAXS <= 2) {
            if (kx < 32 && ky < 32) {
                one_pass = true;
                const bool isy = lane >= 32;
                const int a = lane & 31;
                if (a <= (isy ? ky : kx)) {
                    const float2 e = expm_hw(fixed_mul_hi(isy ? hy : hx, (uint32_t)(a * a)));   // conj(T[+-a])
                    const uint32_t v1 = bf16_pair(e.x, e.y), v2 = bf16_pair(-e.y, e.x);
                    const int c = (isy ? nvyp : nvxp) - 1, len = isy ? tp.ey : tp.ex;
                    uint32_t* t1 = isy ? ty1 : tx1;
                    uint32_t* t2 = isy ? ty2 : tx2;
                    if (c - a >= 0) t1[c - a] = v1, t2[c - a] = v2;
                    if (c + a < len) t1[c + a] = v1, t2[c + a] = v2;
                }
            }
        }
        if (!one_pass) {
            for (int a = lane; a <= kx; a += 64) {
                const float2 e = expm_hw(fixed_mul_hi(hx, (uint32_t)(a * a)));   // conj(Tx[+-a])
                const uint32_t v1 = bf16_pair(e.x, e.y), v2 = bf16_pair(-e.y, e.x);
                const int n1 = nvxp - 1 - a, n2 = nvxp - 1 + a;
                if (n1 >= 0) tx1[n1] = v1, tx2[n1] = v2;
                if (n2 < tp.ex) tx1[n2] = v1, tx2[n2] = v2;
            }
            for (int a = lane; a <= ky; a += 64) {
                const float2 e = expm_hw(fixed_mul_hi(hy, (uint32_t)(a * a)));   // conj(Ty[+-a])
                const uint32_t v1 = bf16_pair(e.x, e.y), v2 = bf16_pair(-e.y, e.x);
                const int n1 = nvyp - 1 - a, n2 = nvyp - 1 + a;
                if (n1 >= 0) ty1[n1] = v1, ty2[n1] = v2;
                if (n2 < tp.ey) ty1[n2] = v1, ty2[n2] = v2;
            }
        }
        // the tables are private to the wave: its LDS writes only have to land before its reads
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();

        u32x4 bc[STREAM ? 1 : MAXS];
#pragma unroll
        for (int t = 0; t < MAXT; ++t) {
            if (t < ntiles) {
                const int ty = t / tiles_x, tx = t - ty * tiles_x;
                if (!STREAM && tx == 0) {
                    // column ivy = 16 ty + r; slot e of step s is chirp m = 16 s + 4 seg + e
                    const uint32_t* pb1 = ty1 + 4 * seg - 16 * ty - r + nvyp - 1;
                    const uint32_t* pb2 = pb1 + tp.ey;
#pragma unroll
                    for (int s = 0; s < MAXS; ++s) {
                        const u32x4 hv = *reinterpret_cast<const u32x4*>(hh + 16 * s + 4 * seg);
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            bc[STREAM ? 0 : s][e] = bf16_pair(dot2_bf16(hv[e], pb1[16 * s + e]),
                                                              dot2_bf16(hv[e], pb2[16 * s + e]));
                    }
                }
                // row ivx = 16 tx + r
                const uint32_t* pa1 = tx1 + 4 * seg - 16 * tx - r + nvxp - 1;
                const uint32_t* pa2 = pa1 + tp.ex;
                f32x4 cr0 = zero4(), ci0 = zero4(), cr1 = zero4(), ci1 = zero4();
                if constexpr (STREAM) {
                    // Mc > 128: the right operand formed step by step (steps is even)
                    const uint32_t* pb1 = ty1 + 4 * seg - 16 * ty - r + nvyp - 1;
                    const uint32_t* pb2 = pb1 + tp.ey;
                    auto step = [&](int o, f32x4& cr, f32x4& ci) {
                        const u32x4 ar = {pa1[o], pa1[o + 1], pa1[o + 2], pa1[o + 3]};
                        const u32x4 ai = {pa2[o], pa2[o + 1], pa2[o + 2], pa2[o + 3]};
                        const u32x4 hv = *reinterpret_cast<const u32x4*>(hh + o + 4 * seg);
                        u32x4 bv;
#pragma unroll
                        for (int e = 0; e < 4; ++e)
                            bv[e] = bf16_pair(dot2_bf16(hv[e], pb1[o + e]), dot2_bf16(hv[e], pb2[o + e]));
                        cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ar), as_bf16x8(bv), cr, 0, 0, 0);
                        ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ai), as_bf16x8(bv), ci, 0, 0, 0);
                    };
                    for (int s2 = 0; s2 < steps; s2 += 2) {
                        step(16 * s2, cr0, ci0);
                        step(16 * s2 + 16, cr1, ci1);
                    }
                } else {
#pragma unroll
                    for (int s = 0; s < MAXS; ++s) {
                        const int o = 16 * s;
                        const u32x4 ar = {pa1[o], pa1[o + 1], pa1[o + 2], pa1[o + 3]};
                        const u32x4 ai = {pa2[o], pa2[o + 1], pa2[o + 2], pa2[o + 3]};
                        // two accumulator pairs in turn; with at most two steps one pair
                        // (saves the pairs' sum, 8 VALU instructions per tile and receiver)
                        f32x4& cr = (MAXS > 2 && (s & 1)) ? cr1 : cr0;
                        f32x4& ci = (MAXS > 2 && (s & 1)) ? ci1 : ci0;
                        cr = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ar), as_bf16x8(bc[s]), cr, 0, 0, 0);
                        ci = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(ai), as_bf16x8(bc[s]), ci, 0, 0, 0);
                    }
                }
                if constexpr (STREAM || MAXS > 2) {
                    cr0 += cr1;
                    ci0 += ci1;
                }
#pragma unroll
                for (int e = 0; e < 4; ++e) dsum[t][e] = fmaf(cr0[e], cr0[e], fmaf(ci0[e], ci0[e], dsum[t][e]));
            }
        }
    }

    slab_peak<MAXT>(dsum, ntiles, tiles_x, nvx, nvy, (int64_t)loc * nv, lane, dec, block, loc, excl, nexcl);
}

// Doppler zoom through chirp tables in FP32 (same factorisation as the BF16
// kernel above, on 16x16x4 FP32 products).  Contraction slot g = 2 kappa + c of
// a product holds the real (c = 0) or imaginary (c = 1) part of chirp
// m = 2 s + kappa at step s, so one product contracts two chirps and a complex
// tile step is two products:
//   left operand, row ivx:   (Re, Im) product forms of Tx[ivx - m],
//                            c = 0: (Re Tx, Im Tx),  c = 1: (-Im Tx, Re Tx);
//   right operand, col ivy:  c = 0: Re(h[m] Ty[ivy - m]),  c = 1: Im(...).
// The wave's LDS holds, per receiver, the tables
//   x0[n] = (Re, Im) Tx[k], x1[n] = (-Im, Re) Tx[k],  k = nvx_pad - 1 - n, n < ex;
//   y0[n] = conj(Ty[k]),    y1[n] = (-Im, Re) conj(Ty[k]),  k = nvy_pad - 1 - n;
//   h[m], m < mcp (zero for m >= Mc),
// each entry n as the pair (v[n], v[n + 2]) in 16 bytes: a lane's indices
// advance by two per step, so one 16-byte read serves two steps (16-byte LDS
// reads move twice the bytes per cycle of 8-byte ones).  A lane reads its
// left operand pair as float2 and forms its right operand as
// Re h y.x + Im h y.y.  STEPS > 0 is the exact step count mcp / 2: the right
// operands of a column tile are formed once, in registers, for all its row
// tiles.  STEPS = 0 forms them step by step, eight steps per loop trip
// (mcp / 2 is a multiple of eight).  h of the next receiver is loaded while the
// current one is in work (Mc <= 128; larger Mc read h per receiver).  Table
// values come from expm_poly.
template <int MAXT, int STEPS>
__global__ __launch_bounds__(kThreads) void direct_doppler_zoom_chirp_f32(Geom g, GridP gp, ToepPlan tp,
                                                                         const float2* __restrict__ hws,
                                                                         float* __restrict__ dec,
                                                                         gh_peak* __restrict__ block,
                                                                         const int64_t* __restrict__ excl, int nexcl) {
    extern __shared__ __attribute__((aligned(16))) float4 toepf_lds[];
    constexpr int kHw = STEPS > 0 ? (2 * STEPS + 63) / 64 : 2;   // h values per lane held ahead
    const int lane = threadIdx.x & 63;
    const int r = lane & 15;
    const int grp = lane >> 4;
    const int kap = grp >> 1, c = grp & 1;
    const int w = threadIdx.x >> 6;
    const int loc = blockIdx.x * (blockDim.x >> 6) + w;
    if (loc >= gp.nloc) return;   // wave-uniform; the kernel has no workgroup barrier
    float4* x0 = toepf_lds + (size_t)w * tp.words;
    float4* x1 = x0 + tp.ex;
    float4* y0 = x1 + tp.ex;
    float4* y1 = y0 + tp.ey;
    float4* hh = y1 + tp.ey;
    const float4* xc = c ? x1 : x0;   // this lane's left-operand table
    const float4* yc = c ? y1 : y0;   // and right-operand table
    const int ix = loc / gp.n[1], iy = loc - ix * gp.n[1];
    const int nvx = gp.n[2], nvy = gp.n[3], nv = gp.nv, mc = g.mc;
    const int nvxp = (nvx + 15) & ~15, nvyp = (nvy + 15) & ~15;
    const int tiles_x = nvxp >> 4, ntiles = tiles_x * (nvyp >> 4);
    const int kx = (nvxp > tp.mcp ? nvxp : tp.mcp) - 1, ky = (nvyp > tp.mcp ? nvyp : tp.mcp) - 1;
    const int steps = STEPS > 0 ? STEPS : tp.mcp >> 1;
    // value v of entry n goes to the low half of pair n and the high half of pair n - 2
    auto put = [](float4* t, int n, float2 v) {
        float2* f = reinterpret_cast<float2*>(t);
        f[2 * n] = v;
        if (n >= 2) f[2 * n - 3] = v;
    };

    float2 hpre[kHw];
    auto load_h = [&](int q) {
        const float2* hq = hws + ((size_t)q * gp.nloc + loc) * mc;
#pragma unroll
        for (int u = 0; u < kHw; ++u) {
            const int m = lane + 64 * u;
            hpre[u] = m < mc ? hq[m] : make_float2(0.f, 0.f);
        }
    };
    const bool pre = STEPS > 0 || tp.mcp <= 64 * kHw;   // else (Mc > 128) h is read per receiver
    if (pre) load_h(0);

    // receiver `lane`: fx / 2 and fy / 2 in 64-bit fixed point
    uint64_t hxl = 0, hyl = 0;
    if (lane < g.k) {
        double rr, wx, wy;
        bistatic(g, lane, gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], rr, wx, wy);
        hxl = cycles_to_fixed64(0.5 * g.fd_per_mps * wx * gp.step[2]);
        hyl = cycles_to_fixed64(0.5 * g.fd_per_mps * wy * gp.step[3]);
    }
    auto bcast64 = [](uint64_t v, int src) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
        return ((uint64_t)hi << 32) | lo;
    };
    auto rhs = [](float4 hv, float4 yv, float& b0, float& b1) {
        b0 = fmaf(hv.x, yv.x, hv.y * yv.y);
        b1 = fmaf(hv.z, yv.z, hv.w * yv.w);
    };

    f32x4 dsum[MAXT];
#pragma unroll
    for (int t = 0; t < MAXT; ++t) dsum[t] = zero4();

    for (int q = 0; q < g.k; ++q) {
        // every lane has finished reading receiver q - 1's tables (in-order LDS per wave)
        __builtin_amdgcn_wave_barrier();
        if (pre) {
#pragma unroll
            for (int u = 0; u < kHw; ++u) {
                const int m = lane + 64 * u;
                if (m < tp.mcp) put(hh, m, hpre[u]);
            }
            if (q + 1 < g.k) load_h(q + 1);
        } else {
            const float2* hq = hws + ((size_t)q * gp.nloc + loc) * mc;
            for (int m = lane; m < tp.mcp; m += 64) put(hh, m, m < mc ? hq[m] : make_float2(0.f, 0.f));
        }
        const uint64_t hx = bcast64(hxl, q), hy = bcast64(hyl, q);
        // the tables are even in k and the tiles read |k| <= max(nv_pad, mcp) - 1:
        // one value per |k|, stored at k and -k
        for (int a = lane; a <= kx; a += 64) {
            const float2 e = expm_poly(fixed_mul_hi(hx, (uint32_t)(a * a)));   // conj(Tx[+-a])
            const float2 v0 = make_float2(e.x, -e.y), v1 = make_float2(e.y, e.x);
            const int n1 = nvxp - 1 - a, n2 = nvxp - 1 + a;
            if (n1 >= 0) put(x0, n1, v0), put(x1, n1, v1);
            if (n2 < tp.ex) put(x0, n2, v0), put(x1, n2, v1);
        }
        for (int a = lane; a <= ky; a += 64) {
            const float2 e = expm_poly(fixed_mul_hi(hy, (uint32_t)(a * a)));   // conj(Ty[+-a])
            const float2 v1 = make_float2(-e.y, e.x);
            const int n1 = nvyp - 1 - a, n2 = nvyp - 1 + a;
            if (n1 >= 0) put(y0, n1, e), put(y1, n1, v1);
            if (n2 < tp.ey) put(y0, n2, e), put(y1, n2, v1);
        }
        // the tables are private to the wave: its LDS writes only have to land before its reads
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        __builtin_amdgcn_wave_barrier();

        float bc[STEPS > 0 ? STEPS : 1];
#pragma unroll
        for (int t = 0; t < MAXT; ++t) {
            if (t < ntiles) {
                const int ty = t / tiles_x, tx = t - ty * tiles_x;
                // column ivy = 16 ty + r, row ivx = 16 tx + r, chirp m = 2 s + kappa at step s:
                // pair 2 s of each table holds steps s and s + 1
                const float4* pb = yc + nvyp - 1 - 16 * ty - r + kap;
                const float4* ph = hh + kap;
                const float4* pa = xc + nvxp - 1 - 16 * tx - r + kap;
                f32x4 cr0 = zero4(), ci0 = zero4(), cr1 = zero4(), ci1 = zero4();
                auto mfma2 = [&](float4 a, float b0, float b1) {
                    cr0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b0, cr0, 0, 0, 0);
                    ci0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b0, ci0, 0, 0, 0);
                    cr1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b1, cr1, 0, 0, 0);
                    ci1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b1, ci1, 0, 0, 0);
                };
                if constexpr (STEPS > 0) {
                    if (tx == 0) {
#pragma unroll
                        for (int s = 0; s < STEPS; s += 2) rhs(ph[2 * s], pb[2 * s], bc[s], bc[s + 1]);
                    }
#pragma unroll
                    for (int s = 0; s < STEPS; s += 2) mfma2(pa[2 * s], bc[s], bc[s + 1]);
                } else {
                    for (int s0 = 0; s0 < steps; s0 += 8) {
#pragma unroll
                        for (int s = s0; s < s0 + 8; s += 2) {
                            float b0, b1;
                            rhs(ph[2 * s], pb[2 * s], b0, b1);
                            mfma2(pa[2 * s], b0, b1);
                        }
                    }
                }
                cr0 += cr1;
                ci0 += ci1;
#pragma unroll
                for (int e = 0; e < 4; ++e) dsum[t][e] = fmaf(cr0[e], cr0[e], fmaf(ci0[e], ci0[e], dsum[t][e]));
            }
        }
    }
    slab_peak<MAXT>(dsum, ntiles, tiles_x, nvx, nvy, (int64_t)loc * nv, lane, dec, block, loc, excl, nexcl);
}

// Launch shape of the chirp-table Doppler zooms: the register bounds they were
// instantiated for (MAXT 4 or 16 tiles; right operands cached for Mc <= 128,
// else formed step by step), and waves per workgroup from the LDS of one table
// set per wave (tp.words words of word_bytes each, at most 64 KB per
// workgroup); waves = 0 when the slab exceeds 16 tiles or one table set
// exceeds 64 KB (then the generating Doppler zoom runs).
struct ChirpShape {
    int maxt, waves;
    bool stream;
};

ChirpShape chirp_shape(const Geom& g, const GridP& gp, int word_bytes) {
    const ToepPlan tp = toep_plan(g.mc, gp.n[2], gp.n[3]);
    const int ntiles = ((gp.n[2] + 15) >> 4) * ((gp.n[3] + 15) >> 4);
    if (ntiles > 16) return {0, 0, false};
    const size_t per_wave = (size_t)tp.words * word_bytes;
    int w = kWaves;
    while (w > 1 && w * per_wave > 65536) w >>= 1;
    if (w * per_wave > 65536) return {0, 0, false};
    return {ntiles <= 4 ? 4 : 16, w, tp.mcp > 128};
}

}  // namespace

size_t direct_ws_bytes(const Geom& g, const GridP& gp, int /*gemm*/) {
    return (size_t)g.k * gp.nloc * g.mc * sizeof(float2);
}

// BF16 range zoom: 16 CT chirps per workgroup (CT = 4 unless Mc < 64), 64 locations.
template <bool CHIRP>
hipError_t launch_range_bf16(const Geom& g, const GridP& gp, const float2* y, void* out, hipStream_t st) {
    const int ct = g.mc >= 64 ? 4 : (g.mc >= 32 ? 2 : 1);
    const dim3 grid((gp.nloc + 16 * kWaves - 1) / (16 * kWaves), (g.mc + 16 * ct - 1) / (16 * ct), g.k);
    if (ct == 4)
        hipLaunchKernelGGL((direct_range_zoom_bf16<1, 4, CHIRP>), grid, dim3(kThreads), 0, st, g, gp, y, out);
    else if (ct == 2)
        hipLaunchKernelGGL((direct_range_zoom_bf16<1, 2, CHIRP>), grid, dim3(kThreads), 0, st, g, gp, y, out);
    else
        hipLaunchKernelGGL((direct_range_zoom_bf16<1, 1, CHIRP>), grid, dim3(kThreads), 0, st, g, gp, y, out);
    return hipGetLastError();
}

hipError_t launch_direct_range(const Geom& g, const GridP& gp, const float2* y, int gemm, float2* G, hipStream_t st) {
    if (gemm == GH_GEMM_BF16) return launch_range_bf16<false>(g, gp, y, G, st);
    const dim3 g1((gp.nloc + 16 * kWaves - 1) / (16 * kWaves), (g.mc + 16 * kNT - 1) / (16 * kNT), g.k);
    hipLaunchKernelGGL(direct_range_zoom, g1, dim3(kThreads), 0, st, g, gp, y, G);
    return hipGetLastError();
}

// Both precisions: the chirp-table Doppler zoom on h from the range zoom when
// its tables fit in LDS, else the generating Doppler zoom on G.  The workspace
// holds G or h (complex64, or BF16 pairs for h in BF16: at most as many bytes).
hipError_t launch_direct(const Geom& g, const GridP& gp, const float2* y, int gemm, void* ws, float* dec,
                         gh_peak* block, const int64_t* excl, int nexcl, hipStream_t st) {
    float2* gws = static_cast<float2*>(ws);
    hipError_t e;
    if (gemm == GH_GEMM_BF16) {
        const ChirpShape cs = chirp_shape(g, gp, 4);
        if (cs.waves > 0) {
            if ((e = launch_range_bf16<true>(g, gp, y, ws, st)) != hipSuccess) return e;
            const ToepPlan tp = toep_plan(g.mc, gp.n[2], gp.n[3]);
            const size_t lds = (size_t)cs.waves * tp.words * 4;
            const dim3 grid((gp.nloc + cs.waves - 1) / cs.waves), blk(64 * cs.waves);
            const uint32_t* h = static_cast<const uint32_t*>(ws);
#define GH_CHIRP_LAUNCH(T, S) \
    hipLaunchKernelGGL((direct_doppler_zoom_chirp<T, S>), grid, blk, lds, st, g, gp, tp, h, dec, block, excl, nexcl)
#define GH_CHIRP_STEPS(T)                                             \
    do {                                                              \
        const int steps = tp.mcp >> 4;   /* 1, 2, 4 or 8 unless streamed */ \
        if (cs.stream) GH_CHIRP_LAUNCH(T, 0);                         \
        else if (steps == 8) GH_CHIRP_LAUNCH(T, 8);                   \
        else if (steps == 4) GH_CHIRP_LAUNCH(T, 4);                   \
        else if (steps == 2) GH_CHIRP_LAUNCH(T, 2);                   \
        else GH_CHIRP_LAUNCH(T, 1);                                   \
    } while (0)
            if (cs.maxt == 4) GH_CHIRP_STEPS(4); else GH_CHIRP_STEPS(16);
#undef GH_CHIRP_STEPS
#undef GH_CHIRP_LAUNCH
        } else {
            if ((e = launch_range_bf16<false>(g, gp, y, ws, st)) != hipSuccess) return e;
            hipLaunchKernelGGL(direct_doppler_zoom<true>, dim3((gp.nloc + kWaves - 1) / kWaves), dim3(kThreads), 0,
                               st, g, gp, gws, dec, block, excl, nexcl);
        }
    } else {
        const ChirpShape cs = chirp_shape(g, gp, 16);
        if (cs.waves > 0) {
            const int nsplit = g.ms >= 128 ? 4 : (g.ms >= 64 ? 2 : 1);
            const int tile_locs = 16 * (kWaves / nsplit);
            const dim3 g1((gp.nloc + tile_locs - 1) / tile_locs, (g.mc + 16 * kNT - 1) / (16 * kNT), g.k);
            hipLaunchKernelGGL(direct_range_zoom_chirp, g1, dim3(kThreads), 0, st, g, gp, y, gws, nsplit);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            const ToepPlan tp = toep_plan(g.mc, gp.n[2], gp.n[3]);
            const size_t lds = (size_t)cs.waves * tp.words * 16;
            const dim3 grid((gp.nloc + cs.waves - 1) / cs.waves), blk(64 * cs.waves);
#define GH_CHIRP_LAUNCH(T, S)                                                                                   \
    hipLaunchKernelGGL((direct_doppler_zoom_chirp_f32<T, S>), grid, blk, lds, st, g, gp, tp, gws, dec, block, excl, \
                       nexcl)
            // right operands cached in registers when a column tile has several row
            // tiles, for up to 4 tiles and Mc <= 128 (a 16-tile instance would not
            // fit), else formed step by step (fewer registers, more waves resident)
            const int steps = tp.mcp >> 1;
            if (cs.maxt == 16 || cs.stream || gp.n[2] <= 16) {
                if (cs.maxt == 4) GH_CHIRP_LAUNCH(4, 0); else GH_CHIRP_LAUNCH(16, 0);
            } else if (steps == 64) {
                GH_CHIRP_LAUNCH(4, 64);
            } else if (steps == 32) {
                GH_CHIRP_LAUNCH(4, 32);
            } else if (steps == 16) {
                GH_CHIRP_LAUNCH(4, 16);
            } else {
                GH_CHIRP_LAUNCH(4, 8);
            }
#undef GH_CHIRP_LAUNCH
        } else {
            if ((e = launch_direct_range(g, gp, y, gemm, gws, st)) != hipSuccess) return e;
            hipLaunchKernelGGL(direct_doppler_zoom<false>, dim3((gp.nloc + kWaves - 1) / kWaves), dim3(kThreads), 0,
                               st, g, gp, gws, dec, block, excl, nexcl);
        }
    }
    return hipGetLastError();
}

}  // namespace gh
