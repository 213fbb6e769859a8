// Block-OMP fit and residual (the multi-target extension the paper names as
// future work, Sec. VI).  Given the support (selected grid cells theta_t), per
// receiver q:
//   least squares  alpha[:, q] = argmin || Y_q - sum_t alpha_t A_q(theta_t) ||^2
//   with the exact atoms A_q(theta) = b(f_d) (x) a(f_r) of eq. (3), through the
//   normal equations  Gram * alpha = A^H Y_q  solved by Cholesky in FP64;
//   Gram[t][u] = <A_u, A_t> = Dir(f_r,u - f_r,t; Ms) * Dir(f_d,u - f_d,t; Mc)
//   with the Dirichlet sum Dir(d; M) = sum_{n<M} exp(j 2 pi d n) in closed form;
//   residual Y_q - sum_t alpha_t A_q(theta_t).
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

__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < kThreads / 64; ++w) t += red[w];
    return t;
}

// One workgroup per receiver: rhs, Gram, Cholesky solve.  Writes alpha
// (complex64 [nsel][K]) and the fixed-point phases of the selected atoms.
__global__ __launch_bounds__(kThreads) void bomp_fit_kernel(Geom g, GridP gp, const float2* __restrict__ y,
                                                           const int64_t* __restrict__ support, int nsel,
                                                           float2* __restrict__ alpha, uint32_t* __restrict__ phases) {
    __shared__ double fr[kMaxSupport], fd[kMaxSupport];
    __shared__ uint32_t frx[kMaxSupport], fdx[kMaxSupport];
    __shared__ dcplx rhs[kMaxSupport];
    __shared__ dcplx gram[kMaxSupport][kMaxSupport];
    __shared__ double red[kThreads / 64];
    const int q = blockIdx.x;
    const int tid = threadIdx.x;
    if (tid < nsel) {
        int64_t idx = support[tid];
        const int ivy = (int)(idx % gp.n[3]);
        idx /= gp.n[3];
        const int ivx = (int)(idx % gp.n[2]);
        idx /= gp.n[2];
        const int iy = (int)(idx % gp.n[1]);
        const int ix = (int)(idx / gp.n[1]);
        double r, wx, wy;
        bistatic(g, q, gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], r, wx, wy);
        const double vx = gp.lo[2] + ivx * gp.step[2], vy = gp.lo[3] + ivy * gp.step[3];
        fr[tid] = g.fr_per_m * r;
        fd[tid] = g.fd_per_mps * (wx * vx + wy * vy);
        frx[tid] = cycles_to_fixed(fr[tid]);
        fdx[tid] = cycles_to_fixed(fd[tid]);
    }
    __syncthreads();
    const float2* yq = y + (size_t)q * g.mc * g.ms;
    const int n = g.mc * g.ms;
    for (int t = 0; t < nsel; ++t) {
        double re = 0.0, im = 0.0;
        const uint32_t a = frx[t], b = fdx[t];
        for (int e = tid; e < n; e += kThreads) {
            const uint32_t m = (uint32_t)(e >> g.log2_ms), s = (uint32_t)(e & (g.ms - 1));
            const float2 ex = expm_fixed(a * s + b * m);
            const float2 v = yq[e];
            re += (double)(v.x * ex.x - v.y * ex.y);
            im += (double)(v.x * ex.y + v.y * ex.x);
        }
        re = block_sum(re, red);
        im = block_sum(im, red);
        if (tid == 0) rhs[t] = {re, im};
    }
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
        dcplx z[kMaxSupport];
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

size_t bomp_fit_ws_bytes(const Geom& g) { return (size_t)kMaxSupport * g.k * 2 * sizeof(uint32_t); }

hipError_t launch_bomp_fit(const Geom& g, const GridP& gp, const float2* y, float2* resid, const int64_t* support,
                           int nsel, float2* alpha, void* ws, hipStream_t st) {
    uint32_t* phases = static_cast<uint32_t*>(ws);
    hipLaunchKernelGGL(bomp_fit_kernel, dim3(g.k), dim3(kThreads), 0, st, g, gp, y, support, nsel, alpha, phases);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int n = g.mc * g.ms;
    hipLaunchKernelGGL(bomp_residual_kernel, dim3((n + kThreads - 1) / kThreads, g.k), dim3(kThreads), 0, st, g, y,
                       resid, alpha, phases, nsel);
    return hipGetLastError();
}

}  // namespace gh
