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
// FP32 products over a chirp, FP64 from there on) and summed in a fixed order;
// the residual's workgroups each solve the small system themselves (identical
// inputs, identical order, so identical alpha), which saves a launch.  They
// also leave the fitted atoms' maps (alpha_t R_t[i] and D_t[l], closed-form
// Dirichlet sums along range and Doppler) for the next selection, whose maps
// of the residual are then the maps of Y minus sum_t alpha_t R_t[i] D_t[l]
// (the maps are linear in the frame).
#include "gh_internal.h"
#include "lane_sum.h"

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
constexpr int kResidWorkgroups = 1024;    // residual grid cap: four workgroups per CU

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
            double pv[2] = {pr, pi};
            group_sum_to_first(pv, 64);   // the wave's sum in lane 0
            if ((tid & 63) == 0) red[tid >> 6][t0 + t] = make_double2(pv[0], pv[1]);
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

// Least squares of receiver q (called by a whole workgroup): sums the
// right-hand side partials, builds the Gram matrix in closed form and solves by
// Cholesky (thread 0, FP64).  Leaves alpha in sh_z and the fixed-point phases
// of the atoms in sh_frx / sh_fdx.
struct FitShared {
    double fr[kMaxSupport], fd[kMaxSupport];
    uint32_t frx[kMaxSupport], fdx[kMaxSupport];
    dcplx rhs[kMaxSupport];
    dcplx gram[kMaxSupport][kMaxSupport];
    dcplx z[kMaxSupport];
};

__device__ void solve_fit(const Geom& g, const GridP& gp, int q, const int64_t* __restrict__ support, int nsel,
                          const double2* __restrict__ part, FitShared& sh) {
    const int tid = threadIdx.x;
    if (tid < nsel) {
        cell_freqs(g, gp, q, support[tid], sh.fr[tid], sh.fd[tid]);
        sh.frx[tid] = cycles_to_fixed(sh.fr[tid]);
        sh.fdx[tid] = cycles_to_fixed(sh.fd[tid]);
        const int nchunk = g.mc / kRowsPerChunk;
        double2 acc = make_double2(0.0, 0.0);
        for (int c = 0; c < nchunk; ++c) {
            const double2 v = part[((size_t)q * nchunk + c) * kMaxSupport + tid];
            acc.x += v.x;
            acc.y += v.y;
        }
        sh.rhs[tid] = {acc.x, acc.y};
    }
    __syncthreads();
    for (int e = tid; e < nsel * nsel; e += blockDim.x) {
        const int t = e / nsel, u = e - t * nsel;
        sh.gram[t][u] = dmul(dirichlet(sh.fr[u] - sh.fr[t], g.ms), dirichlet(sh.fd[u] - sh.fd[t], g.mc));
    }
    __syncthreads();
    if (tid == 0) {
        // Cholesky G = L L^H (lower, in place), then L z = rhs, L^H x = z.
        for (int j = 0; j < nsel; ++j) {
            double d = sh.gram[j][j].x;
            for (int k = 0; k < j; ++k) d -= sh.gram[j][k].x * sh.gram[j][k].x + sh.gram[j][k].y * sh.gram[j][k].y;
            d = sqrt(d > 0.0 ? d : 1e-300);
            sh.gram[j][j] = {d, 0.0};
            for (int i = j + 1; i < nsel; ++i) {
                dcplx s = sh.gram[i][j];
                for (int k = 0; k < j; ++k) {
                    const dcplx p = dconjmul(sh.gram[j][k], sh.gram[i][k]);   // L[i][k] conj(L[j][k])
                    s.x -= p.x;
                    s.y -= p.y;
                }
                sh.gram[i][j] = {s.x / d, s.y / d};
            }
        }
        for (int i = 0; i < nsel; ++i) {
            dcplx s = sh.rhs[i];
            for (int k = 0; k < i; ++k) {
                const dcplx p = dmul(sh.gram[i][k], sh.z[k]);
                s.x -= p.x;
                s.y -= p.y;
            }
            sh.z[i] = {s.x / sh.gram[i][i].x, s.y / sh.gram[i][i].x};
        }
        for (int i = nsel - 1; i >= 0; --i) {
            dcplx s = sh.z[i];
            for (int k = i + 1; k < nsel; ++k) {
                const dcplx p = dconjmul(sh.gram[k][i], sh.z[k]);   // conj(L[k][i]) x[k]
                s.x -= p.x;
                s.y -= p.y;
            }
            sh.z[i] = {s.x / sh.gram[i][i].x, s.y / sh.gram[i][i].x};
        }
    }
    __syncthreads();
}

// sum_{n<M} exp(j 2 pi n (f - idx/N)) * exp(j 2 pi idx c / N), the map value at bin
// idx of a unit tone f along one axis (c: the centring offset, (M - 1)/2 or 0),
// with the Dirichlet sum in closed form: exp(j pi (M - 1) r) sin(pi M r) / sin(pi r),
// r = f - idx/N reduced to [-1/2, 1/2] (the sum has period one in r).  FP64.
__device__ dcplx tone_bin(double f, int m, int n, int idx, double c) {
    const double x = f - (double)idx / n;
    const double r = x - rint(x);
    const double ratio = fabs(r) < 1e-15 ? (double)m : sinpi(m * r) / sinpi(r);
    double sn, cs;
    sincospi((m - 1) * r + 2.0 * idx * c / n, &sn, &cs);
    return {cs * ratio, sn * ratio};
}

// Fit and residual of receiver blockIdx.y: every workgroup solves the (small)
// least squares itself, workgroup 0 also writes alpha (complex64 [nsel][K]), then
//   resid[q][m][s] = y[q][m][s] - sum_t alpha[t][q] exp(+j 2 pi (f_r,t s + f_d,t m)).
__global__ __launch_bounds__(kThreads) void bomp_fit_residual_kernel(Geom g, GridP gp, const float2* __restrict__ y,
                                                                    float2* __restrict__ resid,
                                                                    const int64_t* __restrict__ support, int nsel,
                                                                    const double2* __restrict__ part,
                                                                    float2* __restrict__ alpha,
                                                                    float2* __restrict__ atom_vec) {
    __shared__ FitShared sh;
    __shared__ float2 al[kMaxSupport];
    const int q = blockIdx.y;
    solve_fit(g, gp, q, support, nsel, part, sh);
    if (threadIdx.x < nsel) {
        const float2 a = make_float2((float)sh.z[threadIdx.x].x, (float)sh.z[threadIdx.x].y);
        al[threadIdx.x] = a;
        if (blockIdx.x == 0) alpha[(size_t)threadIdx.x * g.k + q] = a;
    }
    __syncthreads();
    const int n = g.mc * g.ms;
    for (int e = blockIdx.x * kThreads + threadIdx.x; e < n; e += gridDim.x * kThreads) {
        const uint32_t m = (uint32_t)(e >> g.log2_ms), s = (uint32_t)(e & (g.ms - 1));
        float2 v = y[(size_t)q * n + e];
        for (int t = 0; t < nsel; ++t) {
            const float2 em = expm_fixed(sh.frx[t] * s + sh.fdx[t] * m);   // exp(-j ...)
            const float2 at = make_float2(em.x, -em.y);                     // exp(+j ...)
            const float2 a = al[t];
            v.x -= a.x * at.x - a.y * at.y;
            v.y -= a.x * at.y + a.y * at.x;
        }
        resid[(size_t)q * n + e] = v;
    }
    // the maps of each fitted atom of receiver q, alpha_t R_t[i] and D_t[l]
    // (atom_vec[q][t][0 .. N_r) and [N_r .. N_r + N_d)), for the next selection
    const int len = g.nr + g.nd;
    const double cs = g.centered ? 0.5 * (g.ms - 1) : 0.0, cm = g.centered ? 0.5 * (g.mc - 1) : 0.0;
    for (int e = blockIdx.x * kThreads + threadIdx.x; e < nsel * len; e += gridDim.x * kThreads) {
        const int t = e / len, j = e - t * len;
        float2 v;
        if (j < g.nr) {
            const dcplx r = dmul({(double)al[t].x, (double)al[t].y}, tone_bin(sh.fr[t], g.ms, g.nr, j, cs));
            v = make_float2((float)r.x, (float)r.y);
        } else {
            const dcplx d = tone_bin(sh.fd[t], g.mc, g.nd, j - g.nr, cm);
            v = make_float2((float)d.x, (float)d.y);
        }
        atom_vec[((size_t)q * kMaxSupport + t) * len + j] = v;
    }
}

constexpr int kResRows = 2;          // map rows per workgroup of the residual maps
constexpr int kResTable = 4096;      // Doppler-axis values (atoms x N_d) held in LDS

// Row groups of kResRows map rows that each receiver's residual maps need:
// groups first[q], first[q] + 1, ... (modulo N_r / kResRows), count[q] of them.
struct ResRowGroups {
    int first[kMaxRx];
    int count[kMaxRx];
};

// Z_res[q][i][l] = Z_y[q][i][l] - sum_t (alpha_t R_t)[i] D_t[l], where the maps of
// the atom A(theta_t) = b(f_d) (x) a(f_r) are R_t[i] D_t[l] (the single-axis tone
// values above, written by the fit with alpha applied), on the row groups of
// `rg`.  Grid (max_q rg.count[q], K).
__global__ __launch_bounds__(kThreads) void bomp_resid_maps_kernel(Geom g, ResRowGroups rg,
                                                                  const float2* __restrict__ maps_y,
                                                                  const float2* __restrict__ atom_vec, int nsel,
                                                                  float2* __restrict__ out) {
    __shared__ float2 dv[kResTable];
    __shared__ float2 cr[kMaxSupport][kResRows];
    const int q = blockIdx.y, tid = threadIdx.x;
    if ((int)blockIdx.x >= rg.count[q]) return;
    const int ngroups = g.nr / kResRows;
    const int gi = (rg.first[q] + (int)blockIdx.x) % ngroups;
    const int i0 = gi * kResRows;
    const int nd = g.nd, len = g.nr + g.nd;
    const float2* av = atom_vec + (size_t)q * kMaxSupport * len;
    for (int e = tid; e < nsel * nd; e += kThreads) {
        const int t = e >> g.log2_nd, l = e & (nd - 1);
        dv[e] = av[(size_t)t * len + g.nr + l];
    }
    for (int e = tid; e < nsel * kResRows; e += kThreads) {
        const int t = e / kResRows, ii = e - t * kResRows;
        cr[t][ii] = av[(size_t)t * len + i0 + ii];
    }
    __syncthreads();
    const size_t base = ((size_t)q * g.nr + i0) * nd;
    for (int e = tid; e < kResRows * nd; e += kThreads) {
        const int ii = e >> g.log2_nd, l = e & (nd - 1);
        float2 v = maps_y[base + e];
        for (int t = 0; t < nsel; ++t) {
            const float2 c = cr[t][ii], d = dv[t * nd + l];
            v.x -= c.x * d.x - c.y * d.y;
            v.y -= c.x * d.y + c.y * d.x;
        }
        out[base + e] = v;
    }
}

}  // namespace

bool bomp_resid_maps_ok(const Geom& g, int nsel) {
    return nsel >= 1 && nsel <= kMaxSupport && (long)nsel * g.nd <= kResTable && g.nr % kResRows == 0;
}

size_t bomp_atom_vec_bytes(const Geom& g) { return (size_t)g.k * kMaxSupport * (g.nr + g.nd) * sizeof(float2); }

// Map rows the sweep can read for receiver q over the grid's locations: the
// taps floor(t_r) - 1 .. floor(t_r) + 2 (bicubic; bilinear reads a subset) of
// t_r = kr R for R between a lower bound of the bistatic range over the grid's
// (x, y) rectangle (the larger of the baseline and the sum of the two
// distances to the rectangle) and its maximum, which lies at a corner because
// R is convex; one more row on each side covers rounding.  As row groups.
static void touched_row_groups(const Geom& g, const GridP& gp, int q, int& first, int& count) {
    const int ngroups = g.nr / kResRows;
    const double x0 = gp.lo[0], x1 = gp.lo[0] + (gp.n[0] - 1) * gp.step[0];
    const double y0 = gp.lo[1], y1 = gp.lo[1] + (gp.n[1] - 1) * gp.step[1];
    auto to_rect = [&](const double* p) {
        const double dx = fmax(fmax(x0 - p[0], p[0] - x1), 0.0), dy = fmax(fmax(y0 - p[1], p[1] - y1), 0.0);
        return sqrt(dx * dx + dy * dy);
    };
    auto dist = [](double ax, double ay, const double* p) {
        return sqrt((ax - p[0]) * (ax - p[0]) + (ay - p[1]) * (ay - p[1]));
    };
    const double* tx = g.tx;
    const double* rx = g.rx[q];
    double rmax = 0.0;
    for (int c = 0; c < 4; ++c) {
        const double cx = (c & 1) ? x1 : x0, cy = (c & 2) ? y1 : y0;
        rmax = fmax(rmax, dist(cx, cy, tx) + dist(cx, cy, rx));
    }
    const double rmin = fmax(dist(tx[0], tx[1], rx), to_rect(tx) + to_rect(rx));
    const double lo = floor(g.kr * rmin) - 2.0, hi = floor(g.kr * rmax) + 3.0;
    if (!(hi - lo + 1.0 < (double)g.nr)) {
        first = 0;
        count = ngroups;
        return;
    }
    const long long l = (long long)lo, h = (long long)hi;
    const long long gl = (l >= 0 ? l : l - kResRows + 1) / kResRows;   // floor division
    const long long gh = (h >= 0 ? h : h - kResRows + 1) / kResRows;
    count = (int)(gh - gl + 1 < ngroups ? gh - gl + 1 : ngroups);
    first = (int)(((gl % ngroups) + ngroups) % ngroups);
}

hipError_t launch_bomp_resid_maps(const Geom& g, const GridP& gp, const float2* maps_y, const float2* atom_vec,
                                  int nsel, float2* out, hipStream_t st) {
    ResRowGroups rg{};
    int width = 0;
    for (int q = 0; q < g.k; ++q) {
        touched_row_groups(g, gp, q, rg.first[q], rg.count[q]);
        if (rg.count[q] > width) width = rg.count[q];
    }
    hipLaunchKernelGGL(bomp_resid_maps_kernel, dim3(width, g.k), dim3(kThreads), 0, st, g, rg, maps_y, atom_vec, nsel,
                       out);
    return hipGetLastError();
}

size_t bomp_fit_ws_bytes(const Geom& g) {
    return (size_t)g.k * (g.mc / kRowsPerChunk) * kMaxSupport * sizeof(double2);
}

hipError_t launch_bomp_fit(const Geom& g, const GridP& gp, const float2* y, float2* resid, const int64_t* support,
                           int nsel, float2* alpha, void* ws, float2* atom_vec, hipStream_t st) {
    double2* part = static_cast<double2*>(ws);
    hipLaunchKernelGGL(bomp_rhs_kernel, dim3(g.mc / kRowsPerChunk, g.k), dim3(kThreads), 0, st, g, gp, y, support,
                       nsel, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // At most kResidWorkgroups workgroups in all (each holds about 18 KiB of LDS),
    // so the whole grid is resident at once and the solve's latency is paid once.
    const int n = g.mc * g.ms;
    int per_q = (n + kThreads - 1) / kThreads;
    const int cap = kResidWorkgroups / g.k > 0 ? kResidWorkgroups / g.k : 1;
    if (per_q > cap) per_q = cap;
    hipLaunchKernelGGL(bomp_fit_residual_kernel, dim3(per_q, g.k), dim3(kThreads), 0, st, g, gp, y, resid, support,
                       nsel, part, alpha, atom_vec);
    return hipGetLastError();
}

}  // namespace gh
