// Decisions at continuous points and their gradients (the differentiation
// axis; not in the paper): for theta = (x, y, vx, vy),
//   direct:        D = sum_q |c_q|^2, c_q = M_00, moments
//                  M_pq = sum_{m,s} Y_q[m][s] exp(-j 2 pi (f_r s + f_d m)) s^p m^q,
//                  dc_q/dp = -j 2 pi (df_r/dp M_10 + df_d/dp M_01);
//   grid hopping:  D = sum_q |I_q|^2 with the interpolated map value of eq. (7),
//                  dI/dp = N_r dI/dt_r df_r/dp + N_d dI/dt_d df_d/dp,
// and dD/dp = 2 Re(conj(c) dc/dp), for p in theta and in each receiver's
// position (sensing functions of eqs. (1)-(2)).  Frequencies and their
// derivatives are FP64; map taps and sums FP32 per chirp, FP64 beyond.
#include "gh_internal.h"

namespace gh {
namespace {

constexpr int kThreads = 256;
constexpr int kRows = 8;           // chirps per workgroup of the direct moments
constexpr int kTabMax = 1024;      // range phase factors (Ms <= 1024)

struct PtFreq {
    double fr, fd;                 // cycles per sample, per chirp
    double gr[2];                  // d f_r / d(x, y)
    double gd[4];                  // d f_d / d(x, y, vx, vy)
    double rr[2], rd[2];           // d f_r / d rx_q, d f_d / d rx_q
};

// Frequencies of receiver q at theta and their first derivatives.
__device__ void point_freqs(const Geom& g, int q, const double* th, PtFreq& o) {
    const double v0 = th[2], v1 = th[3];
    double rsum = 0.0, w0 = 0.0, w1 = 0.0, j00 = 0.0, j01 = 0.0, j11 = 0.0;
    double q00 = 0.0, q01 = 0.0, q11 = 0.0, qrho = 0.0, u0q = 0.0, u1q = 0.0;
    for (int leg = 0; leg < 2; ++leg) {
        const double ax = leg ? g.rx[q][0] : g.tx[0];
        const double ay = leg ? g.rx[q][1] : g.tx[1];
        const double d0 = th[0] - ax, d1 = th[1] - ay;
        const double rho = sqrt(d0 * d0 + d1 * d1);
        if (rho == 0.0) continue;
        const double u0 = d0 / rho, u1 = d1 / rho;
        rsum += rho;
        w0 += u0;
        w1 += u1;
        j00 += (1.0 - u0 * u0) / rho;
        j01 += -u0 * u1 / rho;
        j11 += (1.0 - u1 * u1) / rho;
        if (leg) {
            q00 = (1.0 - u0 * u0) / rho;
            q01 = -u0 * u1 / rho;
            q11 = (1.0 - u1 * u1) / rho;
            qrho = rho;
            u0q = u0;
            u1q = u1;
        }
    }
    const double br = g.fr_per_m, bd = g.fd_per_mps;
    o.fr = br * rsum;
    o.fd = bd * (w0 * v0 + w1 * v1);
    o.gr[0] = br * w0;
    o.gr[1] = br * w1;
    o.gd[0] = bd * (j00 * v0 + j01 * v1);
    o.gd[1] = bd * (j01 * v0 + j11 * v1);
    o.gd[2] = bd * w0;
    o.gd[3] = bd * w1;
    const bool has = qrho > 0.0;
    o.rr[0] = has ? -br * u0q : 0.0;
    o.rr[1] = has ? -br * u1q : 0.0;
    o.rd[0] = has ? -bd * (q00 * v0 + q01 * v1) : 0.0;
    o.rd[1] = has ? -bd * (q01 * v0 + q11 * v1) : 0.0;
}

// Direct moments M_00, M_10, M_01 of receiver q at point pt over chirps
// [m0, m0 + 8): partials written to part[pt][q][chunk][6] (FP64 re/im).
__global__ __launch_bounds__(kThreads) void direct_points_moments(Geom g, const float2* __restrict__ y,
                                                                 const double* __restrict__ theta,
                                                                 double* __restrict__ part) {
    __shared__ float2 er[kTabMax];
    __shared__ float2 ed[kRows];
    __shared__ uint32_t fx[2];
    __shared__ double red[kThreads / 64][6];
    const int chunk = blockIdx.x, q = blockIdx.y, pt = blockIdx.z;
    const int nchunk = gridDim.x;
    const int tid = threadIdx.x, ms = g.ms;
    const int m0 = chunk * kRows;
    if (tid == 0) {
        PtFreq f;
        point_freqs(g, q, theta + (size_t)pt * 4, f);
        fx[0] = cycles_to_fixed(f.fr);
        fx[1] = cycles_to_fixed(f.fd);
    }
    __syncthreads();
    for (int s = tid; s < ms; s += kThreads) er[s] = expm_fixed(fx[0] * (uint32_t)s);
    if (tid < kRows) ed[tid] = expm_fixed(fx[1] * (uint32_t)(m0 + tid));
    __syncthreads();
    const int tpr = kThreads / kRows;                  // lanes per chirp
    const int row = tid / tpr, lane = tid - row * tpr;
    const float2* yr = y + ((size_t)q * g.mc + m0 + row) * ms;
    float a0r = 0.f, a0i = 0.f, a1r = 0.f, a1i = 0.f;
    for (int s = lane; s < ms; s += tpr) {
        const float2 v = yr[s], e = er[s];
        const float re = fmaf(v.x, e.x, -v.y * e.y), im = fmaf(v.x, e.y, v.y * e.x);
        a0r += re;
        a0i += im;
        a1r = fmaf(re, (float)s, a1r);
        a1i = fmaf(im, (float)s, a1i);
    }
    const float2 d = ed[row];
    const double dm = (double)(m0 + row);
    double acc[6];
    acc[0] = (double)a0r * d.x - (double)a0i * d.y;     // M_00
    acc[1] = (double)a0r * d.y + (double)a0i * d.x;
    acc[2] = (double)a1r * d.x - (double)a1i * d.y;     // M_10
    acc[3] = (double)a1r * d.y + (double)a1i * d.x;
    acc[4] = acc[0] * dm;                                // M_01
    acc[5] = acc[1] * dm;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1)
#pragma unroll
        for (int i = 0; i < 6; ++i) acc[i] += __shfl_xor(acc[i], off, 64);
    if ((tid & 63) == 0)
#pragma unroll
        for (int i = 0; i < 6; ++i) red[tid >> 6][i] = acc[i];
    __syncthreads();
    if (tid < 6) {
        double t = 0.0;
        for (int w = 0; w < kThreads / 64; ++w) t += red[w][tid];
        part[(((size_t)pt * g.k + q) * nchunk + chunk) * 6 + tid] = t;
    }
}

// Sums over receivers of a per-lane (receiver) quantity; lanes >= K hold 0.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One wave per point, one lane per receiver: D, dD/dtheta, dD/drx_q.
__device__ void finish_point(const Geom& g, int pt, int lane, double cr, double ci, double tr_r, double tr_i,
                             double td_r, double td_i, const PtFreq& f, double* value, double* grad,
                             double* grad_rx) {
    // c = cr + j ci; dc/dp = -j 2 pi (df_r/dp (tr_r + j tr_i) + df_d/dp (td_r + j td_i)) with
    // (tr, td) the coefficients multiplying the range and Doppler frequency derivatives
    const double tp = 6.283185307179586;
    const bool on = lane < g.k;
    const double dq = on ? cr * cr + ci * ci : 0.0;
    double gp[4], gx[2];
    for (int a = 0; a < 4; ++a) {
        const double fra = a < 2 ? f.gr[a] : 0.0, fda = f.gd[a];
        const double sr = fra * tr_r + fda * td_r, si = fra * tr_i + fda * td_i;
        // dc = -j tp (sr + j si) = tp si - j tp sr;  2 Re(conj(c) dc) = 2 (cr tp si + ci (-tp sr))
        gp[a] = on ? 2.0 * tp * (cr * si - ci * sr) : 0.0;
    }
    for (int a = 0; a < 2; ++a) {
        const double sr = f.rr[a] * tr_r + f.rd[a] * td_r, si = f.rr[a] * tr_i + f.rd[a] * td_i;
        gx[a] = 2.0 * tp * (cr * si - ci * sr);
    }
    const double dsum = wave_sum(dq);
    double gsum[4];
    for (int a = 0; a < 4; ++a) gsum[a] = wave_sum(gp[a]);
    if (lane == 0) {
        value[pt] = dsum;
        if (grad)
            for (int a = 0; a < 4; ++a) grad[(size_t)pt * 4 + a] = gsum[a];
    }
    if (grad_rx && on) {
        grad_rx[((size_t)pt * g.k + lane) * 2 + 0] = gx[0];
        grad_rx[((size_t)pt * g.k + lane) * 2 + 1] = gx[1];
    }
}

__global__ __launch_bounds__(kThreads) void direct_points_finish(Geom g, int npts, int nchunk,
                                                                const double* __restrict__ theta,
                                                                const double* __restrict__ part,
                                                                double* __restrict__ value, double* __restrict__ grad,
                                                                double* __restrict__ grad_rx) {
    const int lane = threadIdx.x & 63;
    const int pt = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (pt >= npts) return;
    double m[6] = {0, 0, 0, 0, 0, 0};
    PtFreq f{};
    if (lane < g.k) {
        point_freqs(g, lane, theta + (size_t)pt * 4, f);
        const double* src = part + ((size_t)pt * g.k + lane) * nchunk * 6;
        for (int c = 0; c < nchunk; ++c)
            for (int i = 0; i < 6; ++i) m[i] += src[c * 6 + i];
    }
    finish_point(g, pt, lane, m[0], m[1], m[2], m[3], m[4], m[5], f, value, grad, grad_rx);
}

// Keys kernel (a = -1/2) weight and derivative at signed offset d.
__device__ __forceinline__ void keys_wd(double d, double& w, double& dw) {
    const double x = fabs(d), sg = d < 0.0 ? -1.0 : 1.0;
    if (x <= 1.0) {
        w = (1.5 * x - 2.5) * x * x + 1.0;
        dw = sg * (4.5 * x - 5.0) * x;
    } else if (x < 2.0) {
        w = ((-0.5 * x + 2.5) * x - 4.0) * x + 2.0;
        dw = sg * ((-1.5 * x + 5.0) * x - 4.0);
    } else {
        w = 0.0;
        dw = 0.0;
    }
}

template <int DT>
__global__ __launch_bounds__(kThreads) void gh_points_kernel(Geom g, int npts, int interp, const char* __restrict__ maps,
                                                            const double* __restrict__ theta,
                                                            double* __restrict__ value, double* __restrict__ grad,
                                                            double* __restrict__ grad_rx) {
    const int lane = threadIdx.x & 63;
    const int pt = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (pt >= npts) return;
    constexpr int kEs = map_elem_bytes(DT);
    double ir = 0, ii = 0, rr = 0, ri = 0, dr = 0, di = 0;   // I, dI/dt_r, dI/dt_d
    PtFreq f{};
    if (lane < g.k) {
        point_freqs(g, lane, theta + (size_t)pt * 4, f);
        const double tr = f.fr * g.nr, td = f.fd * g.nd;
        const double fr0 = floor(tr), fd0 = floor(td);
        const double a = tr - fr0, b = td - fd0;
        const int ntap = interp ? 4 : 2, off = interp ? -1 : 0;
        double wr[4], dwr[4], wd[4], dwd[4];
        for (int t = 0; t < ntap; ++t) {
            if (interp) {
                keys_wd(a - (t + off), wr[t], dwr[t]);
                keys_wd(b - (t + off), wd[t], dwd[t]);
            } else {
                wr[t] = t ? a : 1.0 - a;
                dwr[t] = t ? 1.0 : -1.0;
                wd[t] = t ? b : 1.0 - b;
                dwd[t] = t ? 1.0 : -1.0;
            }
        }
        const char* mq = maps + (size_t)lane * g.nr * g.nd * kEs;
        const float sc = map_scale(g.ms, g.mc, DT);
        const long long i0 = (long long)fr0 + off, l0 = (long long)fd0 + off;
        for (int u = 0; u < ntap; ++u) {
            const long long ri_ = i0 + u;
            const long long wi = ri_ >= 0 ? ri_ / g.nr : -((-ri_ + g.nr - 1) / g.nr);
            const int row = (int)(ri_ - wi * g.nr);
            const float srow = (wi & 1) ? g.sign_r : 1.f;
            for (int v = 0; v < ntap; ++v) {
                const long long li = l0 + v;
                const long long wl = li >= 0 ? li / g.nd : -((-li + g.nd - 1) / g.nd);
                const int col = (int)(li - wl * g.nd);
                const float s = srow * ((wl & 1) ? g.sign_d : 1.f) * sc;
                const float2 z = map_ld1<DT>(mq, (uint32_t)(((size_t)row * g.nd + col) * kEs));
                const double zr = (double)(z.x * s), zi = (double)(z.y * s);
                const double w = wr[u] * wd[v], wdr = dwr[u] * wd[v], wdd = wr[u] * dwd[v];
                ir += w * zr;
                ii += w * zi;
                rr += wdr * zr;
                ri += wdr * zi;
                dr += wdd * zr;
                di += wdd * zi;
            }
        }
    }
    // dI/dp = N_r dI/dt_r df_r/dp + N_d dI/dt_d df_d/dp; finish_point forms
    // -j 2 pi (df_r/dp T_r + df_d/dp T_d), so T = j N dI/dt / (2 pi)
    const double k2 = 1.0 / 6.283185307179586;
    const double trr = -ri * g.nr * k2, tri = rr * g.nr * k2;
    const double tdr = -di * g.nd * k2, tdi = dr * g.nd * k2;
    finish_point(g, pt, lane, ir, ii, trr, tri, tdr, tdi, f, value, grad, grad_rx);
}

}  // namespace

size_t direct_points_ws_bytes(const Geom& g, int npts) {
    return (size_t)npts * g.k * (g.mc / kRows) * 6 * sizeof(double);
}

hipError_t launch_direct_points(const Geom& g, const float2* y, const double* theta, int npts, void* ws,
                                double* value, double* grad, double* grad_rx, hipStream_t st) {
    double* part = static_cast<double*>(ws);
    const int nchunk = g.mc / kRows;
    hipLaunchKernelGGL(direct_points_moments, dim3(nchunk, g.k, npts), dim3(kThreads), 0, st, g, y, theta, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(direct_points_finish, dim3((npts + 3) / 4), dim3(kThreads), 0, st, g, npts, nchunk, theta,
                       part, value, grad, grad_rx);
    return hipGetLastError();
}

hipError_t launch_gh_points(const Geom& g, const void* maps, int map_dtype, int interp, const double* theta, int npts,
                            double* value, double* grad, double* grad_rx, hipStream_t st) {
    const char* m = static_cast<const char*>(maps);
    const dim3 grid((npts + 3) / 4);
    if (map_dtype == GH_MAP_F16)
        hipLaunchKernelGGL(gh_points_kernel<GH_MAP_F16>, grid, dim3(kThreads), 0, st, g, npts, interp, m, theta, value,
                           grad, grad_rx);
    else if (map_dtype == GH_MAP_BF16)
        hipLaunchKernelGGL(gh_points_kernel<GH_MAP_BF16>, grid, dim3(kThreads), 0, st, g, npts, interp, m, theta,
                           value, grad, grad_rx);
    else
        hipLaunchKernelGGL(gh_points_kernel<GH_MAP_C64>, grid, dim3(kThreads), 0, st, g, npts, interp, m, theta, value,
                           grad, grad_rx);
    return hipGetLastError();
}

}  // namespace gh
