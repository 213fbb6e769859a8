// Block-OMP fit and residual (the multi-target extension the paper names as
// future work, Sec. VI).  Given the support (selected grid cells theta_t), per
// receiver q:
//   least squares  alpha[:, q] = argmin || Y_q - sum_t alpha_t A_q(theta_t) ||^2
//   with the exact atoms A_q(theta) = b(f_d) (x) a(f_r) of eq. (3), through the
//   normal equations  Gram * alpha = A^H Y_q  solved by Cholesky in FP64;
//   Gram[t][u] = <A_u, A_t> = Dir(f_r,u - f_r,t; Ms) * Dir(f_d,u - f_d,t; Mc)
//   with the Dirichlet sum Dir(d; M) = sum_{n<M} exp(j 2 pi d n) in closed form;
//   residual Y_q - sum_t alpha_t A_q(theta_t).
// The right-hand side is spread over workgroups of 8 chirps (separable atoms,
// FP32 products over a chirp, FP64 from there on) and summed in a fixed order.
#include "gh_internal.h"

namespace gh {
namespace {

constexpr int kThreads = 256;

struct dcplx {
    double x, y;
};

__device__ __forceinline__ dcplx dmul(dcplx a, dcplx b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ __forceinline__ dcplx dconjmul(dcplx a, dcplx b) { return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x}; }

// sum_{n<M} exp(j 2 pi d n)
__device__ dcplx dirichlet(double d, int m) {
    const double p = rint(d);
    if (fabs(d - p) < 1e-15) return {(double)m, 0.0};
    const double ratio = sinpi(d * m) / sinpi(d);
    double s, c;
    sincospi(d * (m - 1), &s, &c);
    return {c * ratio, s * ratio};
}

constexpr int kRowsPerChunk = 8;          // chirps per workgroup of the right-hand side
constexpr int kTabEntries = 4096;         // range phase factors per atom group (32 KiB)

// Sensed frequencies (cycles per sample, per chirp) of grid cell idx at receiver q.
__device__ __forceinline__ void cell_freqs(const Geom& g, const GridP& gp, int q, int64_t idx, double& fr, double& fd) {
    const int ivy = (int)(idx % gp.n[3]);
    idx /= gp.n[3];
    const int ivx = (int)(idx % gp.n[2]);
    idx /= gp.n[2];
    const int iy = (int)(idx % gp.n[1]);
    const int ix = (int)(idx / gp.n[1]);
    double r, wx, wy;
    bistatic(g, q, gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], r, wx, wy);
    const double vx = gp.lo[2] + ivx * gp.step[2], vy = gp.lo[3] + ivy * gp.step[3];
    fr = g.fr_per_m * r;
    fd = g.fd_per_mps * (wx * vx + wy * vy);
}

// Right-hand side A^H Y_q over chirps [m0, m0 + 8) of receiver q for every atom,
// using the separable atom: sum_m e_d[m] sum_s Y[m][s] e_r[s].  Writes the
// partial sums part[q][chunk][t] (FP64).
__global__ __launch_bounds__(kThreads) void bomp_rhs_kernel(Geom g, GridP gp, const float2* __restrict__ y,
                                                           const int64_t* __restrict__ support, int nsel,
                                                           double2* __restrict__ part) {
    __shared__ float2 er[kTabEntries];
    __shared__ float2 ed[kMaxSupport][kRowsPerChunk];
    __shared__ uint32_t frx[kMaxSupport], fdx[kMaxSupport];
    __shared__ double2 red[kThreads / 64][kMaxSupport];
    const int q = blockIdx.y, chunk = blockIdx.x;
    const int m0 = chunk * kRowsPerChunk;
    const int tid = threadIdx.x, ms = g.ms;
    if (tid < nsel) {
        double fr, fd;
        cell_freqs(g, gp, q, support[tid], fr, fd);
        frx[tid] = cycles_to_fixed(fr);
        fdx[tid] = cycles_to_fixed(fd);
    }
    __syncthreads();
    for (int e = tid; e < nsel * kRowsPerChunk; e += kThreads) {
        const int t = e / kRowsPerChunk, r = e - t * kRowsPerChunk;
        ed[t][r] = expm_fixed(fdx[t] * (uint32_t)(m0 + r));
    }
    const int tpr = kThreads / kRowsPerChunk;            // lanes per chirp
    const int row = tid / tpr, lane = tid - row * tpr;
    const float2* yr = y + ((size_t)q * g.mc + m0 + row) * ms;
    const int group = kTabEntries / ms;                  // atoms per table fill
    for (int t0 = 0; t0 < nsel; t0 += group) {
        const int na = nsel - t0 < group ? nsel - t0 : group;
        __syncthreads();
        for (int e = tid; e < na * ms; e += kThreads) {
            const int t = e >> g.log2_ms, s = e & (ms - 1);
            er[e] = expm_fixed(frx[t0 + t] * (uint32_t)s);
        }
        __syncthreads();
        for (int t = 0; t < na; ++t) {
            float re = 0.f, im = 0.f;
            for (int s = lane; s < ms; s += tpr) {
                const float2 v = yr[s], e = er[t * ms + s];
                re = fmaf(v.x, e.x, fmaf(-v.y, e.y, re));
                im = fmaf(v.x, e.y, fmaf(v.y, e.x, im));
            }
            const float2 d = ed[t0 + t][row];
            double pr = (double)re * d.x - (double)im * d.y;
            double pi = (double)re * d.y + (double)im * d.x;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) {
                pr += __shfl_xor(pr, off, 64);
                pi += __shfl_xor(pi, off, 64);
            }
            if ((tid & 63) == 0) red[tid >> 6][t0 + t] = make_double2(pr, pi);
        }
    }
    __syncthreads();
    if (tid < nsel) {
        double2 acc = make_double2(0.0, 0.0);
        for (int w = 0; w < kThreads / 64; ++w) {
            acc.x += red[w][tid].x;
            acc.y += red[w][tid].y;
        }
        part[((size_t)q * (g.mc / kRowsPerChunk) + chunk) * kMaxSupport + tid] = acc;
    }
}

// One workgroup per receiver: sums the right-hand side partials, Gram,
// Cholesky solve.  Writes alpha (complex64 [nsel][K]) and the fixed-point
// phases of the selected atoms.
__global__ __launch_bounds__(kThreads) void bomp_fit_kernel(Geom g, GridP gp, const int64_t* __restrict__ support,
                                                           int nsel, const double2* __restrict__ part,
                                                           float2* __restrict__ alpha, uint32_t* __restrict__ phases) {
    __shared__ double fr[kMaxSupport], fd[kMaxSupport];
    __shared__ uint32_t frx[kMaxSupport], fdx[kMaxSupport];
    __shared__ dcplx rhs[kMaxSupport];
    __shared__ dcplx gram[kMaxSupport][kMaxSupport];
    __shared__ dcplx z[kMaxSupport];
    const int q = blockIdx.x;
    const int tid = threadIdx.x;
    if (tid < nsel) {
        cell_freqs(g, gp, q, support[tid], fr[tid], fd[tid]);
        frx[tid] = cycles_to_fixed(fr[tid]);
        fdx[tid] = cycles_to_fixed(fd[tid]);
        const int nchunk = g.mc / kRowsPerChunk;
        double2 acc = make_double2(0.0, 0.0);
        for (int c = 0; c < nchunk; ++c) {
            const double2 v = part[((size_t)q * nchunk + c) * kMaxSupport + tid];
            acc.x += v.x;
            acc.y += v.y;
        }
        rhs[tid] = {acc.x, acc.y};
    }
    __syncthreads();
    for (int e = tid; e < nsel * nsel; e += kThreads) {
        const int t = e / nsel, u = e - t * nsel;
        gram[t][u] = dmul(dirichlet(fr[u] - fr[t], g.ms), dirichlet(fd[u] - fd[t], g.mc));
    }
    __syncthreads();
    if (tid == 0) {
        // Cholesky G = L L^H (lower, in place), then L z = rhs, L^H x = z.
        for (int j = 0; j < nsel; ++j) {
            double d = gram[j][j].x;
            for (int k = 0; k < j; ++k) d -= gram[j][k].x * gram[j][k].x + gram[j][k].y * gram[j][k].y;
            d = sqrt(d > 0.0 ? d : 1e-300);
            gram[j][j] = {d, 0.0};
            for (int i = j + 1; i < nsel; ++i) {
                dcplx s = gram[i][j];
                for (int k = 0; k < j; ++k) {
                    const dcplx p = dconjmul(gram[j][k], gram[i][k]);   // L[i][k] conj(L[j][k])
                    s.x -= p.x;
                    s.y -= p.y;
                }
                gram[i][j] = {s.x / d, s.y / d};
            }
        }
        for (int i = 0; i < nsel; ++i) {
            dcplx s = rhs[i];
            for (int k = 0; k < i; ++k) {
                const dcplx p = dmul(gram[i][k], z[k]);
                s.x -= p.x;
                s.y -= p.y;
            }
            z[i] = {s.x / gram[i][i].x, s.y / gram[i][i].x};
        }
        for (int i = nsel - 1; i >= 0; --i) {
            dcplx s = z[i];
            for (int k = i + 1; k < nsel; ++k) {
                const dcplx p = dconjmul(gram[k][i], z[k]);   // conj(L[k][i]) x[k]
                s.x -= p.x;
                s.y -= p.y;
            }
            z[i] = {s.x / gram[i][i].x, s.y / gram[i][i].x};
        }
        for (int t = 0; t < nsel; ++t) {
            alpha[(size_t)t * g.k + q] = make_float2((float)z[t].x, (float)z[t].y);
            phases[((size_t)t * g.k + q) * 2] = frx[t];
            phases[((size_t)t * g.k + q) * 2 + 1] = fdx[t];
        }
    }
}

// resid[q][m][s] = y[q][m][s] - sum_t alpha[t][q] exp(+j 2 pi (f_r,t s + f_d,t m))
__global__ __launch_bounds__(kThreads) void bomp_residual_kernel(Geom g, const float2* __restrict__ y,
                                                                float2* __restrict__ resid,
                                                                const float2* __restrict__ alpha,
                                                                const uint32_t* __restrict__ phases, int nsel) {
    const int q = blockIdx.y;
    const int n = g.mc * g.ms;
    const int e = blockIdx.x * kThreads + threadIdx.x;
    if (e >= n) return;
    const uint32_t m = (uint32_t)(e >> g.log2_ms), s = (uint32_t)(e & (g.ms - 1));
    float2 v = y[(size_t)q * n + e];
    for (int t = 0; t < nsel; ++t) {
        const size_t o = (size_t)t * g.k + q;
        const float2 em = expm_fixed(phases[2 * o] * s + phases[2 * o + 1] * m);   // exp(-j ...)
        const float2 at = make_float2(em.x, -em.y);                                 // exp(+j ...)
        const float2 al = alpha[o];
        v.x -= al.x * at.x - al.y * at.y;
        v.y -= al.x * at.y + al.y * at.x;
    }
    resid[(size_t)q * n + e] = v;
}

}  // namespace

size_t bomp_fit_ws_bytes(const Geom& g) {
    return (size_t)g.k * (g.mc / kRowsPerChunk) * kMaxSupport * sizeof(double2) +
           (size_t)kMaxSupport * g.k * 2 * sizeof(uint32_t);
}

hipError_t launch_bomp_fit(const Geom& g, const GridP& gp, const float2* y, float2* resid, const int64_t* support,
                           int nsel, float2* alpha, void* ws, hipStream_t st) {
    double2* part = static_cast<double2*>(ws);
    uint32_t* phases = reinterpret_cast<uint32_t*>(part + (size_t)g.k * (g.mc / kRowsPerChunk) * kMaxSupport);
    hipLaunchKernelGGL(bomp_rhs_kernel, dim3(g.mc / kRowsPerChunk, g.k), dim3(kThreads), 0, st, g, gp, y, support,
                       nsel, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(bomp_fit_kernel, dim3(g.k), dim3(kThreads), 0, st, g, gp, support, nsel, part, alpha, phases);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int n = g.mc * g.ms;
    hipLaunchKernelGGL(bomp_residual_kernel, dim3((n + kThreads - 1) / kThreads, g.k), dim3(kThreads), 0, st, g, y,
                       resid, alpha, phases, nsel);
    return hipGetLastError();
}

}  // namespace gh
