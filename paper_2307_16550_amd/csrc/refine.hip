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
// receiver.  Everything is FP64: phases in 64-bit fixed point (cycles, exact
// modulo 1), phase factors by FP64 sincos, products and sums in FP64 (on the
// matrix cores, FP64 tiles).  Near a flat maximum the ascent's decisions
// compare values of D that differ in their 8th digit or beyond, so FP32 sums
// would stop it short of the maximum.  All receivers
// (or as many as the scratch holds) share one pass: their (receiver, chirp)
// rows are spread over the workgroup and reduced by segment.
// Coordinates are scaled by the grid steps (an axis with one grid point is
// held) and kept in the box of +-1 grid step around the cell.  Each iteration
// takes a projected Newton step (Bertsekas, with an epsilon-active set: a
// coordinate next to a face whose gradient points outwards is put on the
// face, the others take the Newton step of the problem restricted to them,
// eigenvalues replaced by -|lambda|); the ascent stops when the projected step
// is below 1e-7 steps in every coordinate (KKT on the box); otherwise the step
// is halved until the decision does not decrease (at most 16 candidates).
// The answer is the converged local maximum of D on the box.

#include <mutex>

#include "gh_internal.h"
#include "lane_sum.h"

namespace gh {
namespace {

constexpr int kThreads = 1024;
constexpr double kTol = 1e-7;
constexpr double kEpsActive = 1e-2;   // cells: widest band next to a face where an outward push puts a coordinate on it


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
        const double s2 = fma(d0, d0, d1 * d1);
        if (s2 == 0.0) continue;
        const double inv = rsqrt_fp64(s2), inv2 = inv * inv;   // 1 / rho, one reciprocal square root per leg
        const double rho = s2 * inv;
        const double u0 = d0 * inv, u1 = d1 * inv;
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
constexpr int kRowsMax = 1024;   // (receiver, chirp) rows per group: one per thread
constexpr int kSegMax = kRowsMax / 16;   // reduction segments per group (at least 16 rows each)

struct Scratch {
    double2 tab[kTab];
    double2 a[3][kRowsMax];      // A_p of each row
    double seg[kSegMax][12];     // per-segment partial moments
    uint64_t frx[kMaxRx], fdx[kMaxRx];
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
        sc.frx[tid] = cycles_to_fixed64(f.fr);
        sc.fdx[tid] = cycles_to_fixed64(f.fd);
    }
    __syncthreads();
    for (int e = tid; e < G * span; e += kThreads) {
        const int qq = e / span, r = e - qq * span;
        sc.tab[e] = (r < ms) ? expm_fixed64(sc.frx[qq] * (uint64_t)r) : expm_fixed64(sc.fdx[qq] * (uint64_t)(r - ms));
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
            const double2* er = sc.tab + qq * span;
#pragma unroll 8
            for (int s = lane; s < ms; s += tpr) {
                const float2 v = yr[s];
                const double2 e = er[s];
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
        const double2 e = sc.tab[qq * span + ms + m];
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

// Contribution of receiver q to the gradient (4) and the upper triangle of
// the Hessian (10, row-major a <= b) of D at theta, from its moments.
__device__ __forceinline__ void newton_terms(const Geom& g, int q, const double th[4], const double* mo,
                                             double out[14]) {
    const double tp = 6.283185307179586;
    FreqC f;
    freq_compact(g, q, th, f);
    double dcr[4], dci[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const double tr = gr_at(f, a) * mo[2] + gd_at(f, a) * mo[4];
        const double ti = gr_at(f, a) * mo[3] + gd_at(f, a) * mo[5];
        dcr[a] = tp * ti;        // -j 2 pi (tr + j ti)
        dci[a] = -tp * tr;
    }
    const double cr = mo[0], ci = mo[1];
    int k = 4;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        out[a] = 2.0 * (cr * dcr[a] + ci * dci[a]);
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
            out[k++] = 2.0 * (dcr[a] * dcr[b] + dci[a] * dci[b] + cr * d2r + ci * d2i);
        }
    }
}

// Projected Newton step in grid-step coordinates z (the box |z_a| <= 1) from
// the summed gradient and Hessian, with an epsilon-active set:
//   w = max_a |clamp(z_a + g_a / L) - z_a| (L: the largest |Hessian diagonal|),
//   eps = min(kEpsActive, w); a free coordinate within eps of a face whose
//   gradient points out of the box is pushed one cell outwards (the clamp of
//   the candidates puts it on the face); on the other free coordinates
//   step = sum_i (e_i . g) / max(|lambda_i|, 1e-12 max|lambda|) e_i over the
//   eigenpairs of the Hessian restricted to them.
// Where that restricted Hessian is negative definite with a moderate condition
// number the step is (-H)^-1 g, solved by Cholesky; otherwise by the cyclic
// Jacobi eigen-decomposition.  A held axis (one grid point) has step 0.
__device__ __forceinline__ void newton_solve(const double t[14], const double h[4], const double z[4],
                                             double step[4]) {
    double gz[4], hz[4][4];
    bool mov[4], push[4];
    int k = 4;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        gz[a] = (h[a] > 0.0) ? t[a] * h[a] : 0.0;
#pragma unroll
        for (int b = a; b < 4; ++b) {
            hz[a][b] = t[k++] * h[a] * h[b];
            hz[b][a] = hz[a][b];
        }
    }
    double curv = 1e-300;
#pragma unroll
    for (int a = 0; a < 4; ++a)
        if (h[a] > 0.0) curv = fmax(curv, fabs(hz[a][a]));
    double w = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) w = fmax(w, fabs(fmin(1.0, fmax(-1.0, z[a] + gz[a] / curv)) - z[a]));
    const double eps = fmin(kEpsActive, w);
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        push[a] = h[a] > 0.0 && ((z[a] >= 1.0 - eps && gz[a] > 0.0) || (z[a] <= -1.0 + eps && gz[a] < 0.0));
        mov[a] = h[a] > 0.0 && !push[a];
    }
    // Cholesky of -H on the moving axes (any other axis gets a unit row and no
    // gradient; its pivot is not part of the definiteness test, whose scale is
    // the moving axes' largest diagonal entry)
    double l[4][4], dmax = 0.0;
    bool spd = true;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) l[a][b] = (mov[a] && mov[b]) ? -hz[a][b] : (a == b ? 1.0 : 0.0);
#pragma unroll
    for (int a = 0; a < 4; ++a)
        if (mov[a]) dmax = fmax(dmax, fabs(l[a][a]));
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        double d = l[j][j];
#pragma unroll
        for (int k2 = 0; k2 < j; ++k2) d -= l[j][k2] * l[j][k2];
        spd = spd && (!mov[j] || d > 1e-10 * dmax);
        const double ljj = sqrt(fmax(d, 1e-300));
        l[j][j] = ljj;
#pragma unroll
        for (int i = j + 1; i < 4; ++i) {
            double v = l[i][j];
#pragma unroll
            for (int k2 = 0; k2 < j; ++k2) v -= l[i][k2] * l[j][k2];
            l[i][j] = v / ljj;
        }
    }
    double gm[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) gm[a] = mov[a] ? gz[a] : 0.0;
    if (spd) {
        double wv[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double v = gm[i];
#pragma unroll
            for (int k2 = 0; k2 < i; ++k2) v -= l[i][k2] * wv[k2];
            wv[i] = v / l[i][i];
        }
#pragma unroll
        for (int i = 3; i >= 0; --i) {
            double v = wv[i];
#pragma unroll
            for (int k2 = i + 1; k2 < 4; ++k2) v -= l[k2][i] * step[k2];
            step[i] = v / l[i][i];
        }
    } else {
        double hm[4][4], vec[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) hm[a][b] = (mov[a] && mov[b]) ? hz[a][b] : 0.0;
        jacobi4(hm, vec);
        double lmax = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) lmax = fmax(lmax, fabs(hm[a][a]));
        const double floor_l = 1e-12 * fmax(lmax, 1e-300);
        double coef[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            double p = 0.0;
#pragma unroll
            for (int a = 0; a < 4; ++a) p += vec[a][i] * gm[a];
            coef[i] = p / fmax(fabs(hm[i][i]), floor_l);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            double s = 0.0;
#pragma unroll
            for (int i = 0; i < 4; ++i) s += vec[a][i] * coef[i];
            step[a] = s;
        }
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) step[a] = push[a] ? (gz[a] > 0.0 ? 1.0 : -1.0) : (mov[a] ? step[a] : 0.0);
}

// Largest component of the projected step clamp(z + step) - z.
__device__ __forceinline__ double projected_step(const double z[4], const double step[4]) {
    double m = 0.0;
#pragma unroll
    for (int a = 0; a < 4; ++a) m = fmax(m, fabs(fmin(1.0, fmax(-1.0, z[a] + step[a])) - z[a]));
    return m;
}

// Newton step from the moments of every receiver (one thread).
__device__ __forceinline__ void newton_step(const Geom& g, const double th[4], const double h[4], const double z[4],
                                            const double (*mom)[12], double step[4]) {
    double t[14];
#pragma unroll
    for (int i = 0; i < 14; ++i) t[i] = 0.0;
    for (int q = 0; q < g.k; ++q) {
        double c[14];
        newton_terms(g, q, th, mom[q], c);
#pragma unroll
        for (int i = 0; i < 14; ++i) t[i] += c[i];
    }
    newton_solve(t, h, z, step);
}

__device__ __forceinline__ void start_point(const GridP& gp, int64_t idx, double th0[4]) {
    const int ivy = (int)(idx % gp.n[3]);
    idx /= gp.n[3];
    const int ivx = (int)(idx % gp.n[2]);
    idx /= gp.n[2];
    const int iy = (int)(idx % gp.n[1]);
    const int ix = (int)(idx / gp.n[1]);
    th0[0] = gp.lo[0] + ix * gp.step[0];
    th0[1] = gp.lo[1] + iy * gp.step[1];
    th0[2] = gp.lo[2] + ivx * gp.step[2];
    th0[3] = gp.lo[3] + ivy * gp.step[3];
}

// Single-workgroup refinement (one workgroup per cell; frames streamed from
// memory).  Used when a cell's cluster would not fit on the device at once.
__global__ __launch_bounds__(kThreads) void refine_single_kernel(Geom g, GridP gp, const float2* __restrict__ y,
                                                                const int64_t* __restrict__ cells, int max_iter,
                                                                double* __restrict__ theta_out) {
    __shared__ Scratch sc;
    __shared__ double mom[kMaxRx][12];
    __shared__ double mom2[kMaxRx][12];
    __shared__ double sh_step[4];
    const int tid = threadIdx.x;
    double th0[4];
    start_point(gp, cells[blockIdx.x], th0);
    const double h[4] = {gp.step[0], gp.step[1], gp.step[2], gp.step[3]};
    double z[4] = {0, 0, 0, 0};
    double d_cur = decision_at(g, y, th0, sc, mom2);
    for (int it = 0; it < max_iter; ++it) {
        double th[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) th[a] = th0[a] + z[a] * h[a];
        {
            const int gs = group_size(g);
            for (int q0 = 0; q0 < g.k; q0 += gs)
                moments_group(g, y, th, q0, (g.k - q0 < gs) ? g.k - q0 : gs, true, sc, mom);
        }
        if (tid == 0) newton_step(g, th, h, z, mom, sh_step);
        __syncthreads();
        double step[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) step[a] = sh_step[a];
        if (projected_step(z, step) < kTol) break;
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

// ---- cluster refinement ------------------------------------------------------
// A cell's (receiver, chirp) rows are split over W workgroups ("the cluster")
// of R rows each.  One pass evaluates all six moments at up to kCand points
// (the line-search candidates z + step/2^i in the order they are tried, or the
// start point): every workgroup reduces its rows of the frame to partial
// moments per receiver, publishes them, meets the rest of the cluster at a
// barrier in global memory and then sums all partials in one fixed order, so
// every workgroup holds bit-identical moments and takes the same decisions (the
// same sequence of passes).  The first acceptable candidate's moments give the
// next Newton step without another pass; the accepted points are those of a
// one-candidate-at-a-time line search.  A launch holds no more workgroups than
// the device keeps resident at once (occupancy times compute units), so on a
// device not shared with other work every workgroup of a cluster is resident
// together; each barrier wait is bounded regardless (an expired wait aborts the
// launch's cells, whose estimates are then NaN).

typedef double f64x4 __attribute__((ext_vector_type(4)));

// C += A B for one 16 x 16 complex tile on the matrix cores (FP64, four real
// 16x16x4 products per complex one).  Lane l = r + 16 g holds the contraction
// indices 8 g + e (e < 8) of row r of A and of column r of B; the output
// element (i, j) is in lane j + 16 (i % 4), slot i / 4 (the FP64 instruction's
// order; its FP32 counterpart keeps four consecutive rows in one lane).
__device__ __forceinline__ void mfma_tile(const double2 (&a)[8], const double2 (&b)[8], f64x4& cre, f64x4& cim) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        cre = __builtin_amdgcn_mfma_f64_16x16x4f64(a[e].x, b[e].x, cre, 0, 0, 0);
        cre = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[e].y, b[e].y, cre, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f64_16x16x4f64(a[e].x, b[e].y, cim, 0, 0, 0);
        cim = __builtin_amdgcn_mfma_f64_16x16x4f64(a[e].y, b[e].x, cim, 0, 0, 0);
    }
}

constexpr int kCT = 512;             // threads of a cluster workgroup
constexpr int kCand = 8;             // points per pass
constexpr int kRowsMaxC = kCT / kCand;   // rows per workgroup (one thread per (point, row))
constexpr int kRowsMinC = kCT / 64;      // at most 64 lanes per row
constexpr int kCandV = 2;            // points per sweep of a row on the VALU path
constexpr int kInFlight = 4;         // frame loads in flight per lane
constexpr int kWgsTarget = 32;       // preferred workgroups per cell
constexpr int kErMax = 4096;         // range phase factors per pass (64 KB of LDS)
constexpr size_t kLdsBytes = 160 * 1024;   // LDS of one workgroup on gfx950
constexpr int kSlotsMax = 4096;      // workgroups per launch (partial-buffer slots)
constexpr unsigned kSpinLimit = 1u << 21;

struct Cluster {
    int rows_per_wg;   // R, a power of two (a divisor or a multiple of Mc)
    int ystage;        // the workgroup's frame rows staged in LDS after the range table (0: read from memory)
    int wgs;           // W = ceil(K Mc / R)
    int slots;         // partial-buffer slots (workgroups of one launch)
    unsigned spin_limit;   // polls before a barrier wait expires
};

struct ClusterShared {
    double2 ed[kCand][kRowsMaxC];         // Doppler phase factor [point][row]
    double2 a[kCand][3][kRowsMaxC];       // A_p [point][p][row]
    double red[kCand][kRowsMaxC / 8][12]; // per-lane-group partial moments
    double mom[kCand][kMaxRx][12];        // the cell's moments at each point of the pass
    double cur[kMaxRx][12];               // moments at the current point
    double terms[kMaxRx][14];             // per-receiver Newton terms
    double tsum[14];
    double th[kCand][4];
    double cand[kCand][4];                // the points in grid-step coordinates
    uint64_t fr[kCand][kMaxRx], fd[kCand][kMaxRx];
    double step[4];
    int ok;
};

// Cluster barrier: arrival count `target` on this cell's counter.  Bounded: a
// wait that exceeds the spin limit, or sees the launch's abort flag, raises the
// flag and returns false (every waiting workgroup then leaves).
__device__ bool cell_barrier(unsigned* ctr, unsigned target, unsigned* abort_flag, unsigned spin_limit, int* ok_sh) {
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        __threadfence();
        atomicAdd(ctr, 1u);
        unsigned spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if (__hip_atomic_load(abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                ++spins > spin_limit) {
                atomicExch(abort_flag, 1u);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(4);
        }
        __threadfence();
        *ok_sh = ok;
    }
    __syncthreads();
    return *ok_sh != 0;
}

struct ClusterCtx {
    int cell, part, slot0, r0, nrows, q_lo, nq;
};

// The matrix-core per-row sums apply when every row of a workgroup belongs to
// one receiver, the rows form 16-row tiles and the samples 32- or 64-sample steps.
// Sample parts of the tiles: as many as the idle waves allow (1, 2 or 4), each
// part a multiple of 32 samples.
__device__ __forceinline__ int mfma_parts(int ntiles, int ms) {
    int kp = 1;
    while (kp < 4 && ntiles * kp * 2 <= kCT / 64 && ms % (32 * kp * 2) == 0) kp *= 2;
    return kp;
}

__device__ __forceinline__ bool mfma_rows(const Cluster& cl, int ms, const ClusterCtx& cx) {
    const int R = cl.rows_per_wg;
    const int ntiles = (R >> 4) * 2;
    return cx.nq == 1 && R % 16 == 0 && ntiles <= kCT / 64 && ms % 32 == 0;
}

// One pass at the points sh.th[0 .. npts): leaves all six moments of every
// receiver at each point in sh.mom.  er: LDS table of range phase factors.
// ysrc: the workgroup's first frame row (in LDS or memory), rows ystride apart.
__device__ bool cluster_pass(const Geom& g, const Cluster& cl, const ClusterCtx& cx, const float2* ysrc, int ystride,
                             double2* er, int npts, unsigned& pass, ClusterShared& sh, unsigned* ctr,
                             unsigned* abort_flag, double* __restrict__ part) {
    const int tid = threadIdx.x;
    const int ms = g.ms, mc = g.mc, R = cl.rows_per_wg;
    if (tid < npts * cx.nq) {
        const int c = tid / cx.nq, i = tid - c * cx.nq;
        FreqC f;
        freq_compact(g, cx.q_lo + i, sh.th[c], f);
        sh.fr[c][i] = cycles_to_fixed64(f.fr);
        sh.fd[c][i] = cycles_to_fixed64(f.fd);
    }
    __syncthreads();
    const int nte = cx.nq * ms;
    // one padded row per point: the matrix-core reads of the eight points' rows at
    // one sample fall in distinct banks
    const int ers = nte + 1;
    for (int e = tid; e < npts * nte; e += kCT) {
        const int c = e / nte, r = e - c * nte;
        const int i = r >> g.log2_ms, s = r & (ms - 1);
        er[c * ers + r] = expm_fixed64(sh.fr[c][i] * (uint64_t)s);
    }
    for (int e = tid; e < npts * cx.nrows; e += kCT) {
        const int c = e / cx.nrows, r = e - c * cx.nrows;
        const int gr = cx.r0 + r;
        sh.ed[c][r] = expm_fixed64(sh.fd[c][(gr >> g.log2_mc) - cx.q_lo] * (uint64_t)(gr & (mc - 1)));
    }
    __syncthreads();
    // per row and point: A_p = sum_s s^p Y[row][s] e_r[s]
    if (npts > 2 && mfma_rows(cl, ms, cx)) {
        // On the matrix cores (passes of more than two points; one or two
        // points take the VALU path below): C[row][col] = sum_s Y[row][s] B[s][col], col = 8 p + c,
        // B[s][col] = s^p e_c[s] (columns 24..31 zero), as 16 x 16 complex tiles.
        // The (R / 16) x 2 tiles go to waves t + ntiles h, h < kparts, each over
        // its part of the samples; part 0 stores, parts 1, 2, ... then add in
        // turn (fixed order).
        const int wave = tid >> 6, lane = tid & 63;
        const int r = lane & 15, grp = lane >> 4;
        const int ntiles = (R >> 4) * 2;
        const int kparts = mfma_parts(ntiles, ms);
        const int h = wave / ntiles, t = wave - h * ntiles;
        const bool active = h < kparts;
        f64x4 cre = {0.0, 0.0, 0.0, 0.0}, cim = {0.0, 0.0, 0.0, 0.0};
        if (active) {
            const int row = (t >> 1) * 16 + r, col = (t & 1) * 16 + r;
            const int pw = col >> 3, c = col & 7;
            const bool rowv = row < cx.nrows, colv = col < 24 && c < npts;
            const float2* yr = ysrc + (size_t)(rowv ? row : 0) * ystride;
            const double2* ec = er + c * ers;
            const int span = ms / kparts;
            for (int s0 = h * span; s0 < (h + 1) * span; s0 += 32) {
                const int sb = s0 + grp * 8;
                double2 a[8], b[8];
                const float4* y4 = reinterpret_cast<const float4*>(yr + sb);
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const float4 v = rowv ? y4[i] : make_float4(0.f, 0.f, 0.f, 0.f);
                    a[2 * i] = make_double2(v.x, v.y);
                    a[2 * i + 1] = make_double2(v.z, v.w);
                }
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const double fs = (double)(sb + e);
                    const double w = pw == 0 ? 1.0 : (pw == 1 ? fs : fs * fs);
                    const double2 ev = colv ? ec[sb + e] : make_double2(0.0, 0.0);
                    b[e] = make_double2(ev.x * w, ev.y * w);
                }
                mfma_tile(a, b, cre, cim);
            }
        }
        const int j = (t & 1) * 16 + r, c_out = j & 7, p_out = j >> 3;
        if (active && h == 0 && j < 24) {
#pragma unroll
            for (int sl = 0; sl < 4; ++sl) sh.a[c_out][p_out][(t >> 1) * 16 + 4 * sl + grp] = make_double2(cre[sl], cim[sl]);
        }
        for (int hh = 1; hh < kparts; ++hh) {
            __syncthreads();
            if (active && h == hh && j < 24) {
#pragma unroll
                for (int sl = 0; sl < 4; ++sl) {
                    double2& d = sh.a[c_out][p_out][(t >> 1) * 16 + 4 * sl + grp];
                    d = make_double2(d.x + cre[sl], d.y + cim[sl]);
                }
            }
        }
    } else {
        // on the VALU: FP64 products and sums, tpr lanes per row, kCandV points per sweep of the row
        const int tpr = kCT / R;
        const int row = tid / tpr, lane = tid & (tpr - 1);
        for (int c0 = 0; c0 < npts; c0 += kCandV) {
            double acc[kCandV][6];
#pragma unroll
            for (int c = 0; c < kCandV; ++c)
#pragma unroll
                for (int i = 0; i < 6; ++i) acc[c][i] = 0.0;
            if (row < cx.nrows) {
                const float2* yr = ysrc + (size_t)row * ystride;
                const int eoff = (((cx.r0 + row) >> g.log2_mc) - cx.q_lo) * ms;
                // kInFlight independent loads per lane, then their products (in sample order)
                for (int s0 = lane; s0 < ms; s0 += kInFlight * tpr) {
                    float2 v[kInFlight];
#pragma unroll
                    for (int k = 0; k < kInFlight; ++k) {
                        const int s = s0 + k * tpr;
                        v[k] = s < ms ? yr[s] : make_float2(0.f, 0.f);
                    }
#pragma unroll
                    for (int k = 0; k < kInFlight; ++k) {
                        const int s = s0 + k * tpr;
                        if (s < ms) {
                            const double fs = (double)s, fs2 = fs * fs;
                            const double vx = v[k].x, vy = v[k].y;
#pragma unroll
                            for (int c = 0; c < kCandV; ++c) {
                                if (c0 + c < npts) {
                                    const double2 e = er[(c0 + c) * ers + eoff + s];
                                    const double re = fma(vx, e.x, -vy * e.y);
                                    const double im = fma(vx, e.y, vy * e.x);
                                    acc[c][0] += re;
                                    acc[c][1] += im;
                                    acc[c][2] = fma(re, fs, acc[c][2]);
                                    acc[c][3] = fma(im, fs, acc[c][3]);
                                    acc[c][4] = fma(re, fs2, acc[c][4]);
                                    acc[c][5] = fma(im, fs2, acc[c][5]);
                                }
                            }
                        }
                    }
                }
            }
            group_sum_to_first(reinterpret_cast<double(&)[kCandV * 6]>(acc), tpr);
            if (lane == 0) {
#pragma unroll
                for (int c = 0; c < kCandV; ++c)
#pragma unroll
                    for (int p = 0; p < 3; ++p)
                        if (c0 + c < npts) sh.a[c0 + c][p][row] = make_double2(acc[c][2 * p], acc[c][2 * p + 1]);
            }
        }
    }
    __syncthreads();
    // per (point, row): Doppler factor and chirp weights, FP64 sums over each receiver's rows
    {
        const int c = tid / R, row = tid - c * R;       // kCand * R <= kCT
        double acc[12];
#pragma unroll
        for (int i = 0; i < 12; ++i) acc[i] = 0.0;
        if (c < npts && row < cx.nrows) {
            const double2 e = sh.ed[c][row];
            const double dm = (double)((cx.r0 + row) & (mc - 1));
#pragma unroll
            for (int p = 0; p < 3; ++p) {
                const double2 a = sh.a[c][p][row];
                const double re = a.x * e.x - a.y * e.y;
                const double im = a.x * e.y + a.y * e.x;
                if (p == 0) {
                    acc[0] = re;
                    acc[1] = im;
                    acc[4] = re * dm;
                    acc[5] = im * dm;
                    acc[10] = re * dm * dm;
                    acc[11] = im * dm * dm;
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
        const int seg = R < mc ? R : mc;               // rows of one receiver in this workgroup
        const int gsz = seg < 64 ? seg : 64;           // of which one lane group of a wave
        group_sum_to_first(acc, gsz);
        if (c < kCand && (row & (gsz - 1)) == 0) {
#pragma unroll
            for (int i = 0; i < 12; ++i) sh.red[c][row / gsz][i] = acc[i];
        }
        __syncthreads();
        const int per = seg / gsz;                     // lane groups per receiver
        const int par = (int)(pass & 1u);
        for (int e = tid; e < npts * cx.nq * 12; e += kCT) {
            const int cc = e / (cx.nq * 12), r = e - cc * (cx.nq * 12);
            const int i = r / 12, k = r - i * 12;
            double t = 0.0;
            for (int j = 0; j < per; ++j) t += sh.red[cc][i * per + j][k];
            part[((((size_t)par * cl.slots + cx.slot0 + cx.part) * kCand + cc) * kMaxRx + i) * 12 + k] = t;
        }
    }
    const bool ok = cell_barrier(ctr + cx.cell, (pass + 1u) * (unsigned)cl.wgs, abort_flag, cl.spin_limit, &sh.ok);
    if (ok) {
        const int par = (int)(pass & 1u);
        const int per_q = R < mc ? mc / R : 1;         // workgroups holding one receiver
        const int q_per = R > mc ? R / mc : 1;         // receivers held by one workgroup
        for (int e = tid; e < npts * g.k * 12; e += kCT) {
            const int c = e / (g.k * 12), r = e - c * (g.k * 12);
            const int q = r / 12, k = r - q * 12;
            double t = 0.0;
            for (int j = 0; j < per_q; ++j) {
                const int p = R < mc ? q * per_q + j : q / q_per;
                const int i = R > mc ? q - p * q_per : 0;
                t += part[((((size_t)par * cl.slots + cx.slot0 + p) * kCand + c) * kMaxRx + i) * 12 + k];
            }
            sh.mom[c][q][k] = t;
        }
    }
    __syncthreads();
    ++pass;
    return ok;
}

__device__ __forceinline__ double point_value(const Geom& g, const double (*mom)[12]) {
    double d = 0.0;
    for (int q = 0; q < g.k; ++q) d += mom[q][0] * mom[q][0] + mom[q][1] * mom[q][1];
    return d;
}

__global__ __launch_bounds__(kCT) void refine_cluster_kernel(Geom g, GridP gp, const float2* __restrict__ y,
                                                            const int64_t* __restrict__ cells, int cell0,
                                                            int max_iter, Cluster cl,
                                                            double* __restrict__ theta_out, unsigned* ctr,
                                                            unsigned* abort_flag, double* part, int* status) {
    extern __shared__ double2 er[];                 // range phase factors of one pass
    __shared__ ClusterShared sh;
    const int tid = threadIdx.x;
    ClusterCtx cx;
    const int lc = (int)blockIdx.x / cl.wgs;        // cell within the launch
    cx.cell = cell0 + lc;
    cx.part = (int)blockIdx.x - lc * cl.wgs;
    cx.slot0 = lc * cl.wgs;
    const int rows = g.k * g.mc;
    cx.r0 = cx.part * cl.rows_per_wg;
    cx.nrows = min(cl.rows_per_wg, rows - cx.r0);
    cx.q_lo = cx.r0 >> g.log2_mc;
    cx.nq = cl.rows_per_wg <= g.mc ? 1 : (cx.nrows + g.mc - 1) >> g.log2_mc;
    // the workgroup's frame rows: read by every pass, so staged once in LDS when they fit
    // (rows padded by 16 bytes: the matrix-core reads of 16 rows fall in distinct banks)
    const float2* ysrc = y + (size_t)cx.r0 * g.ms;
    int ystride = g.ms;
    if (cl.ystage) {
        const int ers = cx.nq * g.ms + 1;
        float2* ys = reinterpret_cast<float2*>(er + kCand * ers);
        ystride = g.ms + 2;
        for (int e = tid; e < cx.nrows * g.ms; e += kCT) {
            const int r = e >> g.log2_ms, s = e & (g.ms - 1);
            ys[r * ystride + s] = ysrc[e];
        }
        ysrc = ys;
    }
    double th0[4];
    start_point(gp, cells[cx.cell], th0);
    const double h[4] = {gp.step[0], gp.step[1], gp.step[2], gp.step[3]};
    double z[4] = {0, 0, 0, 0};
    unsigned pass = 0;
    if (tid < 4) sh.th[0][tid] = th0[tid];
    __syncthreads();
    bool ok = cluster_pass(g, cl, cx, ysrc, ystride, er, 1, pass, sh, ctr, abort_flag, part);
    double d_cur = point_value(g, sh.mom[0]);
    for (int e = tid; e < g.k * 12; e += kCT) sh.cur[e / 12][e % 12] = sh.mom[0][e / 12][e % 12];
    __syncthreads();
    for (int it = 0; ok && it < max_iter; ++it) {
        double th[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) th[a] = th0[a] + z[a] * h[a];
        if (tid < g.k) newton_terms(g, tid, th, sh.cur[tid], sh.terms[tid]);
        __syncthreads();
        if (tid < 14) {
            double t = 0.0;
            for (int q = 0; q < g.k; ++q) t += sh.terms[q][tid];
            sh.tsum[tid] = t;
        }
        __syncthreads();
        if (tid == 0) {
            double t[14];
#pragma unroll
            for (int i = 0; i < 14; ++i) t[i] = sh.tsum[i];
            newton_solve(t, h, z, sh.step);
        }
        __syncthreads();
        double step[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) step[a] = sh.step[a];
        if (projected_step(z, step) < kTol) break;
        int acc_c = -1;
        for (int tries = 0; tries < 16 && acc_c < 0;) {
            const int npts = 16 - tries < kCand ? 16 - tries : kCand;
#pragma unroll
            for (int c = 0; c < kCand; ++c)
#pragma unroll
                for (int a = 0; a < 4; ++a) {
                    const double v = fmin(1.0, fmax(-1.0, z[a] + step[a]));
                    if (tid == 0 && c < npts) {
                        sh.cand[c][a] = v;
                        sh.th[c][a] = th0[a] + v * h[a];
                    }
                    step[a] *= (c < npts) ? 0.5 : 1.0;
                }
            __syncthreads();
            if (!(ok = cluster_pass(g, cl, cx, ysrc, ystride, er, npts, pass, sh, ctr, abort_flag, part))) break;
            for (int c = 0; c < npts; ++c)
                if (point_value(g, sh.mom[c]) >= d_cur) {
                    acc_c = c;
                    break;
                }
            tries += npts;
        }
        if (acc_c < 0) break;
        const double d_new = point_value(g, sh.mom[acc_c]);
        double move = 0.0;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const double v = sh.cand[acc_c][a];
            move = fmax(move, fabs(v - z[a]));
            z[a] = v;
        }
        d_cur = d_new;
        for (int e = tid; e < g.k * 12; e += kCT) sh.cur[e / 12][e % 12] = sh.mom[acc_c][e / 12][e % 12];
        __syncthreads();
        if (move < kTol) break;
    }
    if (cx.part == 0 && tid == 0) {
#pragma unroll
        for (int a = 0; a < 4; ++a) theta_out[(size_t)cx.cell * 4 + a] = ok ? th0[a] + z[a] * h[a] : NAN;
        if (!ok && status) atomicAdd(status, 1);
    }
}

// Zeroes the barrier counters and the abort flag (n words) and the status word.
__global__ void refine_clear_kernel(unsigned* p, int n, int* status) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
    if (i == 0 && status) *status = 0;
}

int pow2_at_least(int v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

Cluster cluster_plan(const Geom& g, int rows_per_wg, int ncells) {
    Cluster cl;
    const int rows = g.k * g.mc;
    cl.rows_per_wg = rows_per_wg;
    cl.ystage = 0;
    cl.wgs = (rows + rows_per_wg - 1) / rows_per_wg;
    const long slots = (long)ncells * cl.wgs;
    cl.slots = (int)(slots < kSlotsMax ? slots : kSlotsMax);
    cl.spin_limit = kSpinLimit;
    return cl;
}

// Largest rows per workgroup: one thread per (point, row), the range phase
// table of the receivers it covers within kErMax, no more than the frame.
int rows_max(const Geom& g) {
    int r = kRowsMaxC;
    while (r > g.mc && (long)kCand * (r / g.mc) * g.ms > kErMax) r >>= 1;
    const int p2 = pow2_at_least(g.k * g.mc);
    if (r > p2) r = p2;
    return r < kRowsMinC ? kRowsMinC : r;
}

// Preferred rows per workgroup: about kWgsTarget workgroups per cell (the
// GH_KNOB_REFINE_ROWS test switch overrides it).
int rows_pref(const Geom& g) {
    int r = pow2_at_least((g.k * g.mc + kWgsTarget - 1) / kWgsTarget);
    if (const int v = knob(GH_KNOB_REFINE_ROWS)) r = v;
    const int hi = rows_max(g);
    if (r > hi) r = hi;
    return r < kRowsMinC ? kRowsMinC : r;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

size_t counters_bytes(int ncells) { return align256(((size_t)ncells + 1) * sizeof(unsigned)); }

}  // namespace

size_t refine_ws_bytes(const Geom& g, int ncells) {
    // the most slots any plan uses: the smallest rows per workgroup
    const Cluster cl = cluster_plan(g, kRowsMinC, ncells);
    return counters_bytes(ncells) + 2 * (size_t)cl.slots * kCand * kMaxRx * 12 * sizeof(double);
}

namespace {

// The launches of one refinement call.  ws: the barrier counters of ncells
// cells and the abort flag (counters_bytes(ncells)), then slots_cap
// partial-buffer slots; cells that need more slots at once than that are
// refined by several launches.
hipError_t launch_refine_slots(const Geom& g, const GridP& gp, const float2* y, const int64_t* cells, int ncells,
                               int max_iter, void* ws, int slots_cap, double* theta, int* status, hipStream_t st) {
    // the one-workgroup-per-cell kernel when the test switch asks for it
    const bool single_only = knob(GH_KNOB_REFINE_SINGLE) != 0;
    int dev = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    // preferred rows per workgroup, doubled while the cells need more than one launch
    Cluster cl{};
    long capacity = 0;
    size_t lds = 0;
    bool found = false;
    for (int r = rows_pref(g); r <= rows_max(g); r <<= 1) {
        Cluster c = cluster_plan(g, r, ncells);
        const int nq = r <= g.mc ? 1 : r / g.mc;
        size_t l = (size_t)kCand * (nq * g.ms + 1) * sizeof(double2);
        if (l > (size_t)(kErMax + kCand) * sizeof(double2)) continue;   // the pass's range table does not fit
        // the frame rows too, within the device's LDS beside the static part
        const size_t ly = (size_t)r * (g.ms + 2) * sizeof(float2);
        c.ystage = (l + ly + sizeof(ClusterShared) + 4096 <= kLdsBytes) ? 1 : 0;   // 4 KB for the rest
        if (c.ystage) l += ly;
        int per_cu = 0;
        if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
                 &per_cu, reinterpret_cast<const void*>(refine_cluster_kernel), kCT, l)) != hipSuccess)
            return e;
        long cap = (long)cus * per_cu;
        if (cap > slots_cap) cap = slots_cap;
        if (cap < c.wgs) continue;
        c.slots = slots_cap;
        cl = c;
        capacity = cap;
        lds = l;
        found = true;
        if ((long)ncells * c.wgs <= cap) break;     // one launch holds every cell
    }
    unsigned* ctr = static_cast<unsigned*>(ws);
    if (single_only || !found) {
        // no barriers: the status is zero
        if (status) {
            hipLaunchKernelGGL(refine_clear_kernel, dim3(1), dim3(64), 0, st, ctr, 0, status);
            if ((e = hipGetLastError()) != hipSuccess) return e;
        }
        hipLaunchKernelGGL(refine_single_kernel, dim3(ncells), dim3(kThreads), 0, st, g, gp, y, cells, max_iter, theta);
        return hipGetLastError();
    }
    const int spin = knob(GH_KNOB_REFINE_SPIN_LIMIT);
    cl.spin_limit = spin > 0 ? (unsigned)spin : kSpinLimit;
    unsigned* abort_flag = ctr + ncells;
    double* part = reinterpret_cast<double*>(static_cast<char*>(ws) + counters_bytes(ncells));
    hipLaunchKernelGGL(refine_clear_kernel, dim3((ncells + 256) / 256), dim3(256), 0, st, ctr, ncells + 1, status);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int batch = (int)(capacity / cl.wgs);
    for (int c0 = 0; c0 < ncells; c0 += batch) {
        const int nb = ncells - c0 < batch ? ncells - c0 : batch;
        Geom ga = g;
        GridP gpa = gp;
        const float2* ya = y;
        const int64_t* ca = cells;
        int c0a = c0, mi = max_iter;
        Cluster cla = cl;
        double* ta = theta;
        int* sa = status;
        void* args[] = {&ga, &gpa, &ya, &ca, &c0a, &mi, &cla, &ta, &ctr, &abort_flag, &part, &sa};
        e = hipLaunchKernel(reinterpret_cast<const void*>(refine_cluster_kernel), dim3(nb * cl.wgs), dim3(kCT), args,
                            lds, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace

hipError_t launch_refine(const Geom& g, const GridP& gp, const float2* y, const int64_t* cells, int ncells,
                         int max_iter, void* ws, double* theta, int* status, hipStream_t st) {
    // the slots refine_ws_bytes sized the workspace for
    return launch_refine_slots(g, gp, y, cells, ncells, max_iter, ws, cluster_plan(g, kRowsMinC, ncells).slots,
                               theta, status, st);
}

// ---- refinement without allocation -----------------------------------------
// Scratch of gh_refine_noalloc: the counters of at most
// GH_REFINE_NOALLOC_MAX_CELLS cells and the abort flag, then as many
// partial-buffer slots (two parities of kCand x kMaxRx x 12 doubles each) as
// the rest holds.  Every device the library runs on holds one copy, at its own
// address, until the process ends; every call on a device shares it.
constexpr size_t kNoAllocBytes = GH_REFINE_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void* scratch_ptr[kMaxDevices] = {};

constexpr size_t kSlotBytes = 2 * (size_t)kCand * kMaxRx * 12 * sizeof(double);

// Device address of the current device's scratch (looked up once per device).
hipError_t noalloc_scratch(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* p = nullptr;
        if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return e;
        scratch_ptr[dev] = p;
    }
    *out = scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

hipError_t launch_refine_noalloc(const Geom& g, const GridP& gp, const float2* y, const int64_t* cells, int ncells,
                                 int max_iter, double* theta, int* status, hipStream_t st) {
    void* ws = nullptr;
    hipError_t e = noalloc_scratch(&ws);
    if (e != hipSuccess) return e;
    // counters first, partials after counters_bytes(ncells) <= counters_bytes(max cells)
    static_assert(kNoAllocBytes > ((size_t)GH_REFINE_NOALLOC_MAX_CELLS + 1) * sizeof(unsigned) + 256 + 64 * kSlotBytes,
                  "the scratch must hold the counters and at least 64 partial-buffer slots");
    const int slots = (int)((kNoAllocBytes - counters_bytes(GH_REFINE_NOALLOC_MAX_CELLS)) / kSlotBytes);
    return launch_refine_slots(g, gp, y, cells, ncells, max_iter, ws, slots, theta, status, st);
}

}  // namespace gh
