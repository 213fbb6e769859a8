// Off-grid refinement of the direct decision (not in the paper; the grid
// estimators stop at a cell).  One workgroup per starting cell runs the whole
// Newton ascent on D(theta) = sum_q |c_q(theta)|^2 in-kernel:
//   c_q = M_00, with moments M_pq = sum_{m,s} Y_q[m][s] E s^p m^q,
//   E = exp(-j 2 pi (f_r s + f_d m)) = e_r[s] e_d[m];
//   dc/da = -j 2 pi (f_r,a M_10 + f_d,a M_01),
//   d2c/da db = -4 pi^2 (f_r,a f_r,b M_20 + (f_r,a f_d,b + f_d,a f_r,b) M_11 + f_d,a f_d,b M_02)
//               - j 2 pi (f_r,ab M_10 + f_d,ab M_01),
// with the analytic derivatives of f_r = B R/(c Ms) and f_d = f0 Tc <w, v>/c
// (eqs. (1)-(2)).  The atom is separable, so the moments are two reductions:
// per chirp A_p[m] = sum_s s^p e_r[s] Y[m][s] (p <= 2), then
// M_pq = sum_m m^q e_d[m] A_p[m]; only Ms + Mc phase factors are evaluated per
// receiver (32-bit fixed-point phases, FP64 accumulation).
// Coordinates are scaled by the grid steps (an axis with one grid point is
// held); the step uses the Hessian's eigenpairs with eigenvalues replaced by
// -|lambda| (cyclic Jacobi, FP64); the ascent stops when every step component
// is below 1e-7 steps; otherwise the step is halved until the decision does
// not decrease (at most 31 candidates) and clamped to +-1 grid step.
#include "gh_internal.h"

namespace gh {
namespace {

constexpr int kThreads = 1024;
constexpr int kWaves = kThreads / 64;
constexpr double kTol = 1e-7;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

struct FreqD {
    double fr, fd;
    double gr[4], gd[4];
    double hr[4][4], hd[4][4];
};

__device__ void freq_derivs(const Geom& g, int q, const double th[4], FreqD& o) {
    const double beta_r = g.fr_per_m, beta_d = g.fd_per_mps;
    double w[2] = {0, 0}, jac[2][2] = {{0, 0}, {0, 0}}, hxx[2][2] = {{0, 0}, {0, 0}}, rsum = 0;
    const double v[2] = {th[2], th[3]};
    for (int leg = 0; leg < 2; ++leg) {
        const double ax = leg ? g.rx[q][0] : g.tx[0];
        const double ay = leg ? g.rx[q][1] : g.tx[1];
        const double d[2] = {th[0] - ax, th[1] - ay};
        const double rho = sqrt(d[0] * d[0] + d[1] * d[1]);
        if (rho == 0.0) continue;
        const double u[2] = {d[0] / rho, d[1] / rho};
        rsum += rho;
        w[0] += u[0];
        w[1] += u[1];
        const double uv = u[0] * v[0] + u[1] * v[1];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                const double delta = (a == b) ? 1.0 : 0.0;
                jac[a][b] += (delta - u[a] * u[b]) / rho;
                hxx[a][b] -= (v[a] * u[b] + u[a] * v[b] + uv * (delta - 3.0 * u[a] * u[b])) / (rho * rho);
            }
    }
    o.fr = beta_r * rsum;
    o.fd = beta_d * (w[0] * v[0] + w[1] * v[1]);
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) o.hr[a][b] = o.hd[a][b] = 0.0;
    o.gr[0] = beta_r * w[0];
    o.gr[1] = beta_r * w[1];
    o.gr[2] = o.gr[3] = 0.0;
    o.gd[0] = beta_d * (jac[0][0] * v[0] + jac[0][1] * v[1]);
    o.gd[1] = beta_d * (jac[1][0] * v[0] + jac[1][1] * v[1]);
    o.gd[2] = beta_d * w[0];
    o.gd[3] = beta_d * w[1];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            o.hr[a][b] = beta_r * jac[a][b];
            o.hd[a][b] = beta_d * hxx[a][b];
            o.hd[a][2 + b] = beta_d * jac[a][b];
            o.hd[2 + b][a] = beta_d * jac[b][a];
        }
}

// Cyclic Jacobi eigen-decomposition of a symmetric 4x4 matrix (a is destroyed:
// its diagonal ends up holding the eigenvalues; v holds eigenvectors as columns).
__device__ void jacobi4(double a[4][4], double v[4][4]) {
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) v[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0, diag = 0.0;
        for (int i = 0; i < 4; ++i) {
            diag += a[i][i] * a[i][i];
            for (int j = i + 1; j < 4; ++j) off += a[i][j] * a[i][j];
        }
        if (off <= 1e-32 * diag || off == 0.0) break;
        for (int p = 0; p < 3; ++p)
            for (int q = p + 1; q < 4; ++q) {
                if (a[p][q] == 0.0) continue;
                const double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < 4; ++k) {
                    const double akp = a[k][p], akq = a[k][q];
                    a[k][p] = c * akp - s * akq;
                    a[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < 4; ++k) {
                    const double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = c * apk - s * aqk;
                    a[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 4; ++k) {
                    const double vkp = v[k][p], vkq = v[k][q];
                    v[k][p] = c * vkp - s * vkq;
                    v[k][q] = s * vkp + c * vkq;
                }
            }
    }
}

constexpr int kChunk = 256;    // chirp rows per stage-A pass

struct Scratch {
    float2 er[1024];           // exp(-j 2 pi f_r s)
    float2 ed[1024];           // exp(-j 2 pi f_d m)
    double2 a[3][kChunk];      // A_p[m] of the current chunk of chirps
    double red[kWaves][12];
};

// Workgroup-wide moments of receiver q at phases (frx, fdx).  full == false:
// only M_00.  Result (12 doubles: re/im of M00, M10, M01, M20, M11, M02)
// broadcast through `out`.
__device__ void moments(const Geom& g, const float2* __restrict__ yq, uint32_t frx, uint32_t fdx, bool full,
                        Scratch& sc, double* out) {
    const int tid = threadIdx.x;
    const int ms = g.ms, mc = g.mc;
    __syncthreads();
    for (int s = tid; s < ms; s += kThreads) sc.er[s] = expm_fixed(frx * (uint32_t)s);
    for (int m = tid; m < mc; m += kThreads) sc.ed[m] = expm_fixed(fdx * (uint32_t)m);
    __syncthreads();
    double acc[12];
    for (int i = 0; i < 12; ++i) acc[i] = 0.0;
    const int rows = mc < kChunk ? mc : kChunk;
    // stage A: `tpr` lanes per chirp row (power of two, at most one wave)
    int tpr = kThreads / rows;
    if (tpr > 64) tpr = 64;
    const int lane = tid & (tpr - 1);
    for (int c0 = 0; c0 < mc; c0 += rows) {
      {
        const int m = c0 + tid / tpr;      // kThreads / tpr >= rows: one pass covers the chunk
        double a0r = 0, a0i = 0, a1r = 0, a1i = 0, a2r = 0, a2i = 0;
        if (tid / tpr < rows) {
            const float2* row = yq + (size_t)m * ms;
            for (int s = lane; s < ms; s += tpr) {
                const float2 v = row[s], e = sc.er[s];
                const double re = (double)v.x * e.x - (double)v.y * e.y;
                const double im = (double)v.x * e.y + (double)v.y * e.x;
                a0r += re;
                a0i += im;
                if (full) {
                    const double ds = (double)s;
                    a1r += re * ds;
                    a1i += im * ds;
                    a2r += re * ds * ds;
                    a2i += im * ds * ds;
                }
            }
        }
        for (int off = tpr >> 1; off >= 1; off >>= 1) {
            a0r += __shfl_xor(a0r, off, 64);
            a0i += __shfl_xor(a0i, off, 64);
            if (full) {
                a1r += __shfl_xor(a1r, off, 64);
                a1i += __shfl_xor(a1i, off, 64);
                a2r += __shfl_xor(a2r, off, 64);
                a2i += __shfl_xor(a2i, off, 64);
            }
        }
        if (tid / tpr < rows && lane == 0) {
            sc.a[0][m - c0] = make_double2(a0r, a0i);
            sc.a[1][m - c0] = make_double2(a1r, a1i);
            sc.a[2][m - c0] = make_double2(a2r, a2i);
        }
      }
      __syncthreads();
      // stage B: sum over the chunk's chirps with the Doppler factors
      if (tid < rows) {
        const int m = c0 + tid;
        const float2 e = sc.ed[m];
        const double dm = (double)m;
        for (int p = 0; p < (full ? 3 : 1); ++p) {
            const double2 a = sc.a[p][tid];
            const double re = a.x * e.x - a.y * e.y;
            const double im = a.x * e.y + a.y * e.x;
            if (p == 0) {
                acc[0] += re;
                acc[1] += im;
                if (full) {
                    acc[4] += re * dm;
                    acc[5] += im * dm;
                    acc[10] += re * dm * dm;
                    acc[11] += im * dm * dm;
                }
            } else if (p == 1) {
                acc[2] += re;
                acc[3] += im;
                acc[8] += re * dm;
                acc[9] += im * dm;
            } else {
                acc[6] += re;
                acc[7] += im;
            }
        }
      }
      __syncthreads();
    }
    const int cnt = full ? 12 : 2;
    for (int i = 0; i < cnt; ++i) {
        const double s = wave_sum(acc[i]);
        if ((tid & 63) == 0) sc.red[tid >> 6][i] = s;
    }
    __syncthreads();
    if (tid < cnt) {
        double t = 0.0;
        for (int w = 0; w < kWaves; ++w) t += sc.red[w][tid];
        out[tid] = t;
    }
    __syncthreads();
}

__device__ double decision_at(const Geom& g, const float2* y, const double th[4], Scratch& sc, double* mom) {
    double dsum = 0.0;
    for (int q = 0; q < g.k; ++q) {
        FreqD fq;
        freq_derivs(g, q, th, fq);
        moments(g, y + (size_t)q * g.mc * g.ms, cycles_to_fixed(fq.fr), cycles_to_fixed(fq.fd), false, sc, mom);
        dsum += mom[0] * mom[0] + mom[1] * mom[1];
    }
    return dsum;
}

__global__ __launch_bounds__(kThreads) void refine_kernel(Geom g, GridP gp, const float2* __restrict__ y,
                                                         const int64_t* __restrict__ cells, int max_iter,
                                                         double* __restrict__ theta_out) {
    __shared__ Scratch sc;
    __shared__ double mom[kMaxRx][12];
    __shared__ double sh_step[4];
    const int tid = threadIdx.x;
    int64_t idx = cells[blockIdx.x];
    const int ivy = (int)(idx % gp.n[3]);
    idx /= gp.n[3];
    const int ivx = (int)(idx % gp.n[2]);
    idx /= gp.n[2];
    const int iy = (int)(idx % gp.n[1]);
    const int ix = (int)(idx / gp.n[1]);
    const double th0[4] = {gp.lo[0] + ix * gp.step[0], gp.lo[1] + iy * gp.step[1], gp.lo[2] + ivx * gp.step[2],
                           gp.lo[3] + ivy * gp.step[3]};
    const double* h = gp.step;
    double z[4] = {0, 0, 0, 0};
    double d_cur = decision_at(g, y, th0, sc, mom[0]);
    const double tp = 6.283185307179586;
    for (int it = 0; it < max_iter; ++it) {
        double th[4];
        for (int a = 0; a < 4; ++a) th[a] = th0[a] + z[a] * h[a];
        for (int q = 0; q < g.k; ++q) {
            FreqD fq;
            freq_derivs(g, q, th, fq);
            moments(g, y + (size_t)q * g.mc * g.ms, cycles_to_fixed(fq.fr), cycles_to_fixed(fq.fd), true, sc,
                    mom[q]);
        }
        if (tid == 0) {
            double grad[4] = {0, 0, 0, 0}, hess[4][4];
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) hess[a][b] = 0.0;
            for (int q = 0; q < g.k; ++q) {
                FreqD f;
                freq_derivs(g, q, th, f);
                const double* mo = mom[q];
                double dcr[4], dci[4];
                for (int a = 0; a < 4; ++a) {
                    const double tr = f.gr[a] * mo[2] + f.gd[a] * mo[4];
                    const double ti = f.gr[a] * mo[3] + f.gd[a] * mo[5];
                    dcr[a] = tp * ti;        // -j 2 pi (tr + j ti)
                    dci[a] = -tp * tr;
                }
                const double cr = mo[0], ci = mo[1];
                for (int a = 0; a < 4; ++a) {
                    grad[a] += 2.0 * (cr * dcr[a] + ci * dci[a]);
                    for (int b = 0; b < 4; ++b) {
                        const double k20 = f.gr[a] * f.gr[b], k11 = f.gr[a] * f.gd[b] + f.gd[a] * f.gr[b];
                        const double k02 = f.gd[a] * f.gd[b];
                        const double pr = k20 * mo[6] + k11 * mo[8] + k02 * mo[10];
                        const double pi = k20 * mo[7] + k11 * mo[9] + k02 * mo[11];
                        const double sr = f.hr[a][b] * mo[2] + f.hd[a][b] * mo[4];
                        const double si = f.hr[a][b] * mo[3] + f.hd[a][b] * mo[5];
                        const double d2r = -tp * tp * pr + tp * si;     // -tp^2 (pr + j pi) - j tp (sr + j si)
                        const double d2i = -tp * tp * pi - tp * sr;
                        hess[a][b] += 2.0 * (dcr[a] * dcr[b] + dci[a] * dci[b] + cr * d2r + ci * d2i);
                    }
                }
            }
            double gz[4], hz[4][4], vec[4][4];
            for (int a = 0; a < 4; ++a) {
                gz[a] = (h[a] > 0.0) ? grad[a] * h[a] : 0.0;
                for (int b = 0; b < 4; ++b) hz[a][b] = hess[a][b] * h[a] * h[b];
            }
            jacobi4(hz, vec);
            double lmax = 0.0;
            for (int a = 0; a < 4; ++a) lmax = fmax(lmax, fabs(hz[a][a]));
            const double floor_l = 1e-12 * fmax(lmax, 1e-300);
            double coef[4];
            for (int i = 0; i < 4; ++i) {
                double p = 0.0;
                for (int a = 0; a < 4; ++a) p += vec[a][i] * gz[a];
                coef[i] = p / fmax(fabs(hz[i][i]), floor_l);
            }
            for (int a = 0; a < 4; ++a) {
                double s = 0.0;
                for (int i = 0; i < 4; ++i) s += vec[a][i] * coef[i];
                sh_step[a] = (h[a] > 0.0) ? s : 0.0;
            }
        }
        __syncthreads();
        double step[4], smax = 0.0;
        for (int a = 0; a < 4; ++a) {
            step[a] = sh_step[a];
            smax = fmax(smax, fabs(step[a]));
        }
        if (smax < kTol) break;
        bool accepted = false;
        double cand[4], d_new = 0.0;
        for (int tries = 0; tries < 31; ++tries) {
            for (int a = 0; a < 4; ++a) cand[a] = fmin(1.0, fmax(-1.0, z[a] + step[a]));
            double thc[4];
            for (int a = 0; a < 4; ++a) thc[a] = th0[a] + cand[a] * h[a];
            d_new = decision_at(g, y, thc, sc, mom[0]);
            if (d_new >= d_cur) {
                accepted = true;
                break;
            }
            for (int a = 0; a < 4; ++a) step[a] *= 0.5;
        }
        if (!accepted) break;
        double move = 0.0;
        for (int a = 0; a < 4; ++a) {
            move = fmax(move, fabs(cand[a] - z[a]));
            z[a] = cand[a];
        }
        d_cur = d_new;
        if (move < kTol) break;
    }
    if (tid == 0)
        for (int a = 0; a < 4; ++a) theta_out[(size_t)blockIdx.x * 4 + a] = th0[a] + z[a] * h[a];
}

}  // namespace

hipError_t launch_refine(const Geom& g, const GridP& gp, const float2* y, const int64_t* cells, int ncells,
                         int max_iter, double* theta, hipStream_t st) {
    hipLaunchKernelGGL(refine_kernel, dim3(ncells), dim3(kThreads), 0, st, g, gp, y, cells, max_iter, theta);
    return hipGetLastError();
}

}  // namespace gh
