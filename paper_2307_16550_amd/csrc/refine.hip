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
// receiver (32-bit fixed-point phases, FP64 accumulation).  All receivers
// (or as many as the scratch holds) share one pass: their (receiver, chirp)
// rows are spread over the workgroup and reduced by segment.
// Coordinates are scaled by the grid steps (an axis with one grid point is
// held); the step uses the Hessian's eigenpairs with eigenvalues replaced by
// -|lambda| (cyclic Jacobi, FP64); the ascent stops when every step component
// is below 1e-7 steps; otherwise the step is halved until the decision does
// not decrease (at most 16 candidates) and clamped to +-1 grid step.
#include "gh_internal.h"

namespace gh {
namespace {

constexpr int kThreads = 1024;
constexpr double kTol = 1e-7;

// f_r, f_d and their first and second derivatives, kept to the structurally
// nonzero entries: f_r depends on (x, y) only, f_d is linear in v, and
// d2 f_d / dx dv = beta_d J with J symmetric.
struct FreqC {
    double fr, fd;
    double gr0, gr1;                 // d f_r / d(x, y)
    double gd0, gd1, gd2, gd3;       // d f_d / d(x, y, vx, vy)
    double hr00, hr01, hr11;         // d2 f_r / dx dx
    double hd00, hd01, hd11;         // d2 f_d / dx dx
    double hj00, hj01, hj11;         // d2 f_d / dx dv
};

__device__ __forceinline__ double gr_at(const FreqC& f, int a) { return a == 0 ? f.gr0 : (a == 1 ? f.gr1 : 0.0); }
__device__ __forceinline__ double gd_at(const FreqC& f, int a) {
    return a == 0 ? f.gd0 : (a == 1 ? f.gd1 : (a == 2 ? f.gd2 : f.gd3));
}
__device__ __forceinline__ double hr_at(const FreqC& f, int a, int b) {
    if (a > 1 || b > 1) return 0.0;
    return a != b ? f.hr01 : (a == 0 ? f.hr00 : f.hr11);
}
__device__ __forceinline__ double hd_at(const FreqC& f, int a, int b) {
    if (a < 2 && b < 2) return a != b ? f.hd01 : (a == 0 ? f.hd00 : f.hd11);
    if (a >= 2 && b >= 2) return 0.0;
    const int i = a < 2 ? a : b, j = (a < 2 ? b : a) - 2;
    return i != j ? f.hj01 : (i == 0 ? f.hj00 : f.hj11);
}

__device__ __forceinline__ void freq_compact(const Geom& g, int q, const double th[4], FreqC& o) {
    const double beta_r = g.fr_per_m, beta_d = g.fd_per_mps;
    double w0 = 0, w1 = 0, j00 = 0, j01 = 0, j11 = 0, x00 = 0, x01 = 0, x11 = 0, rsum = 0;
    const double v0 = th[2], v1 = th[3];
#pragma unroll
    for (int leg = 0; leg < 2; ++leg) {
        const double ax = leg ? g.rx[q][0] : g.tx[0];
        const double ay = leg ? g.rx[q][1] : g.tx[1];
        const double d0 = th[0] - ax, d1 = th[1] - ay;
        const double rho = sqrt(d0 * d0 + d1 * d1);
        if (rho == 0.0) continue;
        const double u0 = d0 / rho, u1 = d1 / rho, inv = 1.0 / rho, inv2 = inv * inv;
        const double uv = u0 * v0 + u1 * v1;
        rsum += rho;
        w0 += u0;
        w1 += u1;
        j00 += (1.0 - u0 * u0) * inv;
        j01 += -u0 * u1 * inv;
        j11 += (1.0 - u1 * u1) * inv;
        x00 -= (2.0 * v0 * u0 + uv * (1.0 - 3.0 * u0 * u0)) * inv2;
        x01 -= (v0 * u1 + u0 * v1 - uv * 3.0 * u0 * u1) * inv2;
        x11 -= (2.0 * v1 * u1 + uv * (1.0 - 3.0 * u1 * u1)) * inv2;
    }
    o.fr = beta_r * rsum;
    o.fd = beta_d * (w0 * v0 + w1 * v1);
    o.gr0 = beta_r * w0;
    o.gr1 = beta_r * w1;
    o.gd0 = beta_d * (j00 * v0 + j01 * v1);
    o.gd1 = beta_d * (j01 * v0 + j11 * v1);
    o.gd2 = beta_d * w0;
    o.gd3 = beta_d * w1;
    o.hr00 = beta_r * j00;
    o.hr01 = beta_r * j01;
    o.hr11 = beta_r * j11;
    o.hd00 = beta_d * x00;
    o.hd01 = beta_d * x01;
    o.hd11 = beta_d * x11;
    o.hj00 = beta_d * j00;
    o.hj01 = beta_d * j01;
    o.hj11 = beta_d * j11;
}

// Cyclic Jacobi eigen-decomposition of a symmetric 4x4 matrix (a is destroyed:
// its diagonal ends up holding the eigenvalues; v holds eigenvectors as columns).
__device__ __forceinline__ void jacobi4(double a[4][4], double v[4][4]) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) v[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 50; ++sweep) {
        double off = 0.0, diag = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            diag += a[i][i] * a[i][i];
#pragma unroll
            for (int j = i + 1; j < 4; ++j) off += a[i][j] * a[i][j];
        }
        if (off <= 1e-32 * diag || off == 0.0) break;
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = p + 1; q < 4; ++q) {
                if (a[p][q] == 0.0) continue;
                const double theta = (a[q][q] - a[p][p]) / (2.0 * a[p][q]);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const double akp = a[k][p], akq = a[k][q];
                    a[k][p] = c * akp - s * akq;
                    a[k][q] = s * akp + c * akq;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const double apk = a[p][k], aqk = a[q][k];
                    a[p][k] = c * apk - s * aqk;
                    a[q][k] = s * apk + c * aqk;
                }
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const double vkp = v[k][p], vkq = v[k][q];
                    v[k][p] = c * vkp - s * vkq;
                    v[k][q] = s * vkp + c * vkq;
                }
            }
    }
}

constexpr int kTab = 3072;       // phase factors of one receiver group (e_r then e_d per receiver)
constexpr int kRowsMax = 512;    // (receiver, chirp) rows per group
constexpr int kSegMax = 64;      // reduction segments per group

struct Scratch {
    float2 tab[kTab];
    double2 a[3][kRowsMax];      // A_p of each row
    double seg[kSegMax][12];     // per-segment partial moments
    uint32_t frx[kMaxRx], fdx[kMaxRx];
};

// Receivers per pass: the group's phase tables and rows must fit the scratch.
__device__ __forceinline__ int group_size(const Geom& g) {
    int gs = kTab / (g.ms + g.mc);
    const int by_rows = kRowsMax / g.mc;
    if (by_rows < gs) gs = by_rows;
    if (gs > g.k) gs = g.k;
    return gs < 1 ? 1 : gs;
}

// Workgroup-wide moments of receivers [q0, q0 + G) at theta, all in one pass:
// out[q][0..11] = re/im of M00, M10, M01, M20, M11, M02 (full) or M00 only.
__device__ __forceinline__ void moments_group(const Geom& g, const float2* __restrict__ y, const double th[4], int q0, int G,
                              bool full, Scratch& sc, double (*out)[12]) {
    const int tid = threadIdx.x;
    const int ms = g.ms, mc = g.mc, span = ms + mc;
    if (tid < G) {
        FreqC f;
        freq_compact(g, q0 + tid, th, f);
        sc.frx[tid] = cycles_to_fixed(f.fr);
        sc.fdx[tid] = cycles_to_fixed(f.fd);
    }
    __syncthreads();
    for (int e = tid; e < G * span; e += kThreads) {
        const int qq = e / span, r = e - qq * span;
        sc.tab[e] = (r < ms) ? expm_fixed(sc.frx[qq] * (uint32_t)r) : expm_fixed(sc.fdx[qq] * (uint32_t)(r - ms));
    }
    __syncthreads();
    // stage A: tpr lanes per (receiver, chirp) row, sums over fast time
    const int rows = G * mc;
    int tpr = 1;
    while (tpr * 2 * rows <= kThreads && tpr < 64) tpr *= 2;
    const int lane = tid & (tpr - 1);
    const int row = tid / tpr;
    {
        double a0r = 0, a0i = 0, a1r = 0, a1i = 0, a2r = 0, a2i = 0;
        if (row < rows) {
            const int qq = row / mc, m = row - qq * mc;
            const float2* yr = y + ((size_t)(q0 + qq) * mc + m) * ms;
            const float2* er = sc.tab + qq * span;
#pragma unroll 8
            for (int s = lane; s < ms; s += tpr) {
                const float2 v = yr[s], e = er[s];
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
        if (row < rows && lane == 0) {
            sc.a[0][row] = make_double2(a0r, a0i);
            sc.a[1][row] = make_double2(a1r, a1i);
            sc.a[2][row] = make_double2(a2r, a2i);
        }
    }
    __syncthreads();
    // stage B: Doppler factors, then a segmented reduction over each receiver's chirps
    double acc[12];
    for (int i = 0; i < 12; ++i) acc[i] = 0.0;
    if (tid < rows) {
        const int qq = tid / mc, m = tid - qq * mc;
        const float2 e = sc.tab[qq * span + ms + m];
        const double dm = (double)m;
        for (int p = 0; p < (full ? 3 : 1); ++p) {
            const double2 a = sc.a[p][tid];
            const double re = a.x * e.x - a.y * e.y;
            const double im = a.x * e.y + a.y * e.x;
            if (p == 0) {
                acc[0] = re;
                acc[1] = im;
                if (full) {
                    acc[4] = re * dm;
                    acc[5] = im * dm;
                    acc[10] = re * dm * dm;
                    acc[11] = im * dm * dm;
                }
            } else if (p == 1) {
                acc[2] = re;
                acc[3] = im;
                acc[8] = re * dm;
                acc[9] = im * dm;
            } else {
                acc[6] = re;
                acc[7] = im;
            }
        }
    }
    const int cnt = full ? 12 : 2;
    const int seg = mc < 64 ? mc : 64;                // rows of one receiver are contiguous and wave-aligned
    for (int i = 0; i < cnt; ++i)
        for (int off = seg >> 1; off >= 1; off >>= 1) acc[i] += __shfl_xor(acc[i], off, 64);
    if (tid < rows && (tid & (seg - 1)) == 0)
        for (int i = 0; i < cnt; ++i) sc.seg[tid / seg][i] = acc[i];
    __syncthreads();
    const int per_q = mc / seg;
    if (tid < G * cnt) {
        const int qq = tid / cnt, c = tid - qq * cnt;
        double t = 0.0;
        for (int i = 0; i < per_q; ++i) t += sc.seg[qq * per_q + i][c];
        out[q0 + qq][c] = t;
    }
    __syncthreads();
}

__device__ __forceinline__ double decision_at(const Geom& g, const float2* y, const double th[4], Scratch& sc, double (*mom)[12]) {
    const int gs = group_size(g);
    for (int q0 = 0; q0 < g.k; q0 += gs) moments_group(g, y, th, q0, (g.k - q0 < gs) ? g.k - q0 : gs, false, sc, mom);
    double dsum = 0.0;
    for (int q = 0; q < g.k; ++q) dsum += mom[q][0] * mom[q][0] + mom[q][1] * mom[q][1];
    return dsum;
}

__global__ __launch_bounds__(kThreads) void refine_kernel(Geom g, GridP gp, const float2* __restrict__ y,
                                                         const int64_t* __restrict__ cells, int max_iter,
                                                         double* __restrict__ theta_out) {
    __shared__ Scratch sc;
    __shared__ double mom[kMaxRx][12];
    __shared__ double mom2[kMaxRx][12];
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
    double d_cur = decision_at(g, y, th0, sc, mom2);
    const double tp = 6.283185307179586;
    for (int it = 0; it < max_iter; ++it) {
        double th[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) th[a] = th0[a] + z[a] * h[a];
        {
            const int gs = group_size(g);
            for (int q0 = 0; q0 < g.k; q0 += gs)
                moments_group(g, y, th, q0, (g.k - q0 < gs) ? g.k - q0 : gs, true, sc, mom);
        }
        if (tid == 0) {
            double grad[4] = {0, 0, 0, 0}, hess[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) hess[a][b] = 0.0;
            for (int q = 0; q < g.k; ++q) {
                FreqC f;
                freq_compact(g, q, th, f);
                const double* mo = mom[q];
                double dcr[4], dci[4];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const double tr = gr_at(f, a) * mo[2] + gd_at(f, a) * mo[4];
                    const double ti = gr_at(f, a) * mo[3] + gd_at(f, a) * mo[5];
                    dcr[a] = tp * ti;        // -j 2 pi (tr + j ti)
                    dci[a] = -tp * tr;
                }
                const double cr = mo[0], ci = mo[1];
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    grad[a] += 2.0 * (cr * dcr[a] + ci * dci[a]);
#pragma unroll
                    for (int b = a; b < 4; ++b) {
                        const double k20 = gr_at(f, a) * gr_at(f, b);
                        const double k11 = gr_at(f, a) * gd_at(f, b) + gd_at(f, a) * gr_at(f, b);
                        const double k02 = gd_at(f, a) * gd_at(f, b);
                        const double pr = k20 * mo[6] + k11 * mo[8] + k02 * mo[10];
                        const double pi = k20 * mo[7] + k11 * mo[9] + k02 * mo[11];
                        const double sr = hr_at(f, a, b) * mo[2] + hd_at(f, a, b) * mo[4];
                        const double si = hr_at(f, a, b) * mo[3] + hd_at(f, a, b) * mo[5];
                        const double d2r = -tp * tp * pr + tp * si;     // -tp^2 (pr + j pi) - j tp (sr + j si)
                        const double d2i = -tp * tp * pi - tp * sr;
                        hess[a][b] += 2.0 * (dcr[a] * dcr[b] + dci[a] * dci[b] + cr * d2r + ci * d2i);
                    }
                }
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < a; ++b) hess[a][b] = hess[b][a];
            double gz[4], hz[4][4], vec[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                gz[a] = (h[a] > 0.0) ? grad[a] * h[a] : 0.0;
#pragma unroll
                for (int b = 0; b < 4; ++b) hz[a][b] = hess[a][b] * h[a] * h[b];
            }
            jacobi4(hz, vec);
            double lmax = 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a) lmax = fmax(lmax, fabs(hz[a][a]));
            const double floor_l = 1e-12 * fmax(lmax, 1e-300);
            double coef[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                double p = 0.0;
#pragma unroll
                for (int a = 0; a < 4; ++a) p += vec[a][i] * gz[a];
                coef[i] = p / fmax(fabs(hz[i][i]), floor_l);
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                double s = 0.0;
#pragma unroll
                for (int i = 0; i < 4; ++i) s += vec[a][i] * coef[i];
                sh_step[a] = (h[a] > 0.0) ? s : 0.0;
            }
        }
        __syncthreads();
        double step[4], smax = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            step[a] = sh_step[a];
            smax = fmax(smax, fabs(step[a]));
        }
        if (smax < kTol) break;
        bool accepted = false;
        double cand[4], d_new = 0.0;
        for (int tries = 0; tries < 16; ++tries) {
#pragma unroll
            for (int a = 0; a < 4; ++a) cand[a] = fmin(1.0, fmax(-1.0, z[a] + step[a]));
            double thc[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) thc[a] = th0[a] + cand[a] * h[a];
            d_new = decision_at(g, y, thc, sc, mom2);
            if (d_new >= d_cur) {
                accepted = true;
                break;
            }
#pragma unroll
            for (int a = 0; a < 4; ++a) step[a] *= 0.5;
        }
        if (!accepted) break;
        double move = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            move = fmax(move, fabs(cand[a] - z[a]));
            z[a] = cand[a];
        }
        d_cur = d_new;
        if (move < kTol) break;
    }
    if (tid == 0)
#pragma unroll
        for (int a = 0; a < 4; ++a) theta_out[(size_t)blockIdx.x * 4 + a] = th0[a] + z[a] * h[a];
}

}  // namespace

hipError_t launch_refine(const Geom& g, const GridP& gp, const float2* y, const int64_t* cells, int ncells,
                         int max_iter, double* theta, hipStream_t st) {
    hipLaunchKernelGGL(refine_kernel, dim3(ncells), dim3(kThreads), 0, st, g, gp, y, cells, max_iter, theta);
    return hipGetLastError();
}

}  // namespace gh
