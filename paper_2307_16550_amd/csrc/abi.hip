// C ABI of the grid-hopping library: host-side validation, derived radar
// constants, workspace carving and dispatch to the gfx950 kernels.  Nothing is
// enqueued unless every argument has been checked; errors are reported as a
// gh_status plus a thread-local message, never as an exception.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <initializer_list>

#include "gh_internal.h"

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return code;
}

int ok() {
    g_err[0] = '\0';
    return GH_OK;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(GH_EHIP, "%s: %s", what, hipGetErrorString(e));
}

bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

int ilog2(int v) {
    int l = 0;
    while ((1 << l) < v) ++l;
    return l;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

int check_device() {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "no usable HIP device");
    return GH_OK;
}

int make_geom(const gh_radar* r, gh::Geom& g) {
    if (!r) return fail(GH_EINVAL, "radar is NULL");
    if (!finite_pos(r->f0_hz) || !finite_pos(r->bandwidth_hz) || !finite_pos(r->t_chirp_s) || !finite_pos(r->c_mps))
        return fail(GH_EINVAL, "f0, bandwidth, chirp duration and c must be positive and finite");
    if (!pow2(r->n_samples) || r->n_samples < 8 || r->n_samples > 1024)
        return fail(GH_EINVAL, "n_samples must be a power of two in [8, 1024] (got %d)", r->n_samples);
    if (!pow2(r->n_chirps) || r->n_chirps < 8 || r->n_chirps > 1024)
        return fail(GH_EINVAL, "n_chirps must be a power of two in [8, 1024] (got %d)", r->n_chirps);
    if (!pow2(r->pad_range) || r->pad_range > 8 || !pow2(r->pad_doppler) || r->pad_doppler > 8)
        return fail(GH_EINVAL, "pad_range and pad_doppler must be 1, 2, 4 or 8");
    const long nr = (long)r->pad_range * r->n_samples, nd = (long)r->pad_doppler * r->n_chirps;
    if (nr > 4096 || nd > 4096) return fail(GH_EINVAL, "map sizes N_r = %ld, N_d = %ld exceed 4096", nr, nd);
    if (r->n_rx < 1 || r->n_rx > GH_MAX_RX) return fail(GH_EINVAL, "n_rx must be in [1, %d]", GH_MAX_RX);
    if (r->centered != 0 && r->centered != 1) return fail(GH_EINVAL, "centered must be 0 or 1");
    if (!r->rx) return fail(GH_EINVAL, "rx is NULL");
    if (!isfinite(r->tx[0]) || !isfinite(r->tx[1])) return fail(GH_EINVAL, "tx is not finite");
    memset(&g, 0, sizeof(g));
    g.tx[0] = r->tx[0];
    g.tx[1] = r->tx[1];
    for (int q = 0; q < r->n_rx; ++q) {
        if (!isfinite(r->rx[2 * q]) || !isfinite(r->rx[2 * q + 1])) return fail(GH_EINVAL, "rx[%d] is not finite", q);
        g.rx[q][0] = r->rx[2 * q];
        g.rx[q][1] = r->rx[2 * q + 1];
    }
    g.k = r->n_rx;
    g.ms = r->n_samples;
    g.mc = r->n_chirps;
    g.pr = r->pad_range;
    g.pd = r->pad_doppler;
    g.nr = (int)nr;
    g.nd = (int)nd;
    g.log2_ms = ilog2(g.ms);
    g.log2_mc = ilog2(g.mc);
    g.log2_nr = ilog2(g.nr);
    g.log2_nd = ilog2(g.nd);
    g.centered = r->centered;
    g.sign_r = (r->centered && (g.ms % 2 == 0)) ? -1.f : 1.f;
    g.sign_d = (r->centered && (g.mc % 2 == 0)) ? -1.f : 1.f;
    g.kr = r->bandwidth_hz * r->pad_range / r->c_mps;
    g.kd = r->f0_hz * r->t_chirp_s * r->pad_doppler * r->n_chirps / r->c_mps;
    g.fr_per_m = r->bandwidth_hz / (r->c_mps * r->n_samples);
    g.fd_per_mps = r->f0_hz * r->t_chirp_s / r->c_mps;
    return GH_OK;
}

int make_grid(const gh_grid* gr, gh::GridP& gp) {
    if (!gr) return fail(GH_EINVAL, "grid is NULL");
    long long total = 1;
    for (int a = 0; a < 4; ++a) {
        if (gr->n[a] < 1) return fail(GH_EINVAL, "grid axis %d has n = %d < 1", a, gr->n[a]);
        if (!isfinite(gr->lo[a]) || !isfinite(gr->hi[a]) || gr->lo[a] > gr->hi[a])
            return fail(GH_EINVAL, "grid axis %d needs finite lo <= hi", a);
        total *= gr->n[a];
        gp.lo[a] = gr->lo[a];
        gp.step[a] = (gr->n[a] == 1) ? 0.0 : (gr->hi[a] - gr->lo[a]) / (gr->n[a] - 1);
        gp.n[a] = gr->n[a];
    }
    if (total >= (1LL << 31)) return fail(GH_EINVAL, "grid has %lld points (limit 2^31 - 1)", total);
    gp.nloc = gr->n[0] * gr->n[1];
    gp.nv = gr->n[2] * gr->n[3];
    if (gp.nv > 4096) return fail(GH_EUNSUPPORTED, "velocity slab Nvx*Nvy = %d exceeds 4096", gp.nv);
    return GH_OK;
}

// The sweep keeps one receiver's Doppler table and profile in LDS.
int check_sweep_limits(const gh::Geom& g, int interp) {
    if (interp != GH_INTERP_BILINEAR && interp != GH_INTERP_BICUBIC)
        return fail(GH_EINVAL, "interp must be GH_INTERP_BILINEAR or GH_INTERP_BICUBIC");
    const size_t lds = (size_t)g.nd * (interp ? 32 : 16) + (size_t)g.nd * 8;
    if (lds > 65536) return fail(GH_EUNSUPPORTED, "N_d = %d too large for the %s sweep", g.nd, interp ? "bicubic" : "bilinear");
    return GH_OK;
}

int check_gemm(int gemm) {
    if (gemm != GH_GEMM_F32 && gemm != GH_GEMM_BF16) return fail(GH_EINVAL, "gemm_dtype must be F32 or BF16");
    return GH_OK;
}

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// The half storage formats park complex64 range spectra in their rows, which
// needs N_d * 4 >= Mc * 8 bytes.
int check_map_dtype(const gh::Geom& g, int dt) {
    if (dt != GH_MAP_C64 && dt != GH_MAP_F16 && dt != GH_MAP_BF16)
        return fail(GH_EINVAL, "map_dtype must be GH_MAP_C64, GH_MAP_F16 or GH_MAP_BF16");
    if (dt != GH_MAP_C64 && g.pd < 2) return fail(GH_EUNSUPPORTED, "16-bit map storage needs pad_doppler >= 2");
    return GH_OK;
}

// Device arrays are read and written with 16-byte vector accesses.
int check_aligned(std::initializer_list<const void*> ptrs) {
    for (const void* p : ptrs)
        if (((uintptr_t)p & 15) != 0) return fail(GH_EINVAL, "device arrays must be 16-byte aligned");
    return GH_OK;
}

}  // namespace

extern "C" {

int gh_abi_version(void) { return GH_ABI_VERSION; }

const char* gh_last_error(void) { return g_err; }

int gh_rd_maps(const gh_radar* radar, const void* d_y, void* d_maps, int32_t map_dtype, void* stream) {
    gh::Geom g;
    int rc = make_geom(radar, g);
    if (rc || (rc = check_map_dtype(g, map_dtype))) return rc;
    if (!d_y || !d_maps) return fail(GH_EINVAL, "d_y and d_maps must be non-NULL");
    if ((rc = check_aligned({d_y, d_maps}))) return rc;
    const size_t ybytes = (size_t)g.k * g.mc * g.ms * 8,
                 mbytes = (size_t)g.k * g.nr * g.nd * gh::map_elem_bytes(map_dtype);
    const char *y0 = (const char*)d_y, *m0 = (const char*)d_maps;
    if (y0 < m0 + mbytes && m0 < y0 + ybytes) return fail(GH_EINVAL, "d_y and d_maps overlap");
    if ((rc = check_device())) return rc;
    hipError_t e = gh::launch_rd_maps(g, (const float2*)d_y, d_maps, map_dtype, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gh_rd_maps launch");
    return ok();
}

int gh_decision(const gh_radar* radar, const gh_grid* grid, const void* d_maps, int32_t map_dtype, int32_t interp,
                float* d_decision, gh_peak* d_block, gh_peak* d_argmax, void* stream) {
    gh::Geom g;
    gh::GridP gp;
    int rc = make_geom(radar, g);
    if (rc || (rc = make_grid(grid, gp)) || (rc = check_sweep_limits(g, interp)) || (rc = check_map_dtype(g, map_dtype)))
        return rc;
    if (!d_maps || !d_block) return fail(GH_EINVAL, "d_maps and d_block must be non-NULL");
    if ((rc = check_aligned({d_maps, d_decision, d_block, d_argmax}))) return rc;
    if ((rc = check_device())) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = gh::launch_gh_sweep(g, gp, d_maps, map_dtype, interp, d_decision, d_block, nullptr, 0, st);
    if (e == hipSuccess && d_argmax) e = gh::launch_peak_final(d_block, gp.nloc, d_argmax, nullptr, st);
    if (e != hipSuccess) return hip_fail(e, "gh_decision launch");
    return ok();
}

int gh_argmax(const gh_peak* d_block, int64_t n_block, gh_peak* d_argmax, void* stream) {
    if (!d_block || !d_argmax) return fail(GH_EINVAL, "d_block and d_argmax must be non-NULL");
    if (n_block < 1 || n_block >= (1LL << 31)) return fail(GH_EINVAL, "n_block must be in [1, 2^31)");
    int rc = check_aligned({d_block, d_argmax});
    if (rc || (rc = check_device())) return rc;
    hipError_t e = gh::launch_peak_final(d_block, (int)n_block, d_argmax, nullptr, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gh_argmax launch");
    return ok();
}

size_t gh_direct_workspace_bytes(const gh_radar* radar, const gh_grid* grid, int32_t gemm_dtype) {
    gh::Geom g;
    gh::GridP gp;
    if (make_geom(radar, g) || make_grid(grid, gp) || check_gemm(gemm_dtype)) return 0;
    ok();
    return align256(gh::direct_ws_bytes(g, gp, gemm_dtype));
}

int gh_direct_decision(const gh_radar* radar, const gh_grid* grid, const void* d_y, int32_t gemm_dtype, void* d_ws,
                       size_t ws_bytes, float* d_decision, gh_peak* d_block, gh_peak* d_argmax, void* stream) {
    gh::Geom g;
    gh::GridP gp;
    int rc = make_geom(radar, g);
    if (rc || (rc = make_grid(grid, gp)) || (rc = check_gemm(gemm_dtype))) return rc;
    if (!d_y || !d_block || !d_ws) return fail(GH_EINVAL, "d_y, d_ws and d_block must be non-NULL");
    if ((rc = check_aligned({d_y, d_ws, d_decision, d_block, d_argmax}))) return rc;
    const size_t need = align256(gh::direct_ws_bytes(g, gp, gemm_dtype));
    if (ws_bytes < need) return fail(GH_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((rc = check_device())) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = gh::launch_direct(g, gp, (const float2*)d_y, gemm_dtype, d_ws, d_decision, d_block, nullptr, 0, st);
    if (e == hipSuccess && d_argmax) e = gh::launch_peak_final(d_block, gp.nloc, d_argmax, nullptr, st);
    if (e != hipSuccess) return hip_fail(e, "gh_direct_decision launch");
    return ok();
}

size_t gh_bomp_workspace_bytes(const gh_radar* radar, const gh_grid* grid, int32_t use_direct, int32_t gemm_dtype) {
    gh::Geom g;
    gh::GridP gp;
    if (make_geom(radar, g) || make_grid(grid, gp) || check_gemm(gemm_dtype)) return 0;
    ok();
    size_t b = align256((size_t)gp.nloc * sizeof(gh_peak)) + align256(gh::bomp_fit_ws_bytes(g));
    if (use_direct) b += align256(gh::direct_ws_bytes(g, gp, gemm_dtype));
    return b;
}

int gh_bomp_step(const gh_radar* radar, const gh_grid* grid, const void* d_y, void* d_resid, void* d_maps,
                 int32_t use_direct, int32_t interp, int32_t gemm_dtype, int64_t* d_support, int32_t n_support,
                 int32_t max_support, void* d_alpha, gh_peak* d_selected, void* d_ws, size_t ws_bytes, void* stream) {
    gh::Geom g;
    gh::GridP gp;
    int rc = make_geom(radar, g);
    if (rc || (rc = make_grid(grid, gp)) || (rc = check_gemm(gemm_dtype))) return rc;
    if (use_direct != 0 && use_direct != 1) return fail(GH_EINVAL, "use_direct must be 0 or 1");
    if (!use_direct && (rc = check_sweep_limits(g, interp))) return rc;
    if (!d_y || !d_resid || !d_support || !d_alpha || !d_ws) return fail(GH_EINVAL, "NULL device pointer");
    if (!use_direct && !d_maps) return fail(GH_EINVAL, "d_maps must be non-NULL for grid hopping");
    if ((rc = check_aligned({d_y, d_resid, d_maps, d_support, d_alpha, d_selected, d_ws}))) return rc;
    if (max_support < 1 || max_support > GH_MAX_SUPPORT)
        return fail(GH_EINVAL, "max_support must be in [1, %d]", GH_MAX_SUPPORT);
    if (n_support < 0 || n_support >= max_support)
        return fail(GH_EINVAL, "n_support = %d must be in [0, max_support)", n_support);
    if (n_support + 1 > gp.nloc * (long long)gp.nv) return fail(GH_EINVAL, "support larger than the grid");
    const size_t need = gh_bomp_workspace_bytes(radar, grid, use_direct, gemm_dtype);
    if (ws_bytes < need) return fail(GH_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((rc = check_device())) return rc;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    gh_peak* block = (gh_peak*)ws;
    ws += align256((size_t)gp.nloc * sizeof(gh_peak));
    void* fit_ws = ws;
    ws += align256(gh::bomp_fit_ws_bytes(g));
    void* dir_ws = ws;
    hipError_t e;
    if (use_direct) {
        e = gh::launch_direct(g, gp, (const float2*)d_resid, gemm_dtype, dir_ws, nullptr, block, d_support, n_support, st);
    } else {
        e = gh::launch_rd_maps(g, (const float2*)d_resid, d_maps, GH_MAP_C64, st);
        if (e == hipSuccess)
            e = gh::launch_gh_sweep(g, gp, d_maps, GH_MAP_C64, interp, nullptr, block, d_support, n_support, st);
    }
    if (e == hipSuccess) e = gh::launch_peak_final(block, gp.nloc, d_selected, d_support + n_support, st);
    if (e == hipSuccess)
        e = gh::launch_bomp_fit(g, gp, (const float2*)d_y, (float2*)d_resid, d_support, n_support + 1,
                                (float2*)d_alpha, fit_ws, st);
    if (e != hipSuccess) return hip_fail(e, "gh_bomp_step launch");
    return ok();
}

size_t gh_refine_workspace_bytes(const gh_radar* radar, const gh_grid* grid, int32_t n_cells) {
    gh::Geom g;
    gh::GridP gp;
    if (make_geom(radar, g) || make_grid(grid, gp)) return 0;
    if (n_cells < 1 || n_cells > 65535) {
        fail(GH_EINVAL, "n_cells must be in [1, 65535]");
        return 0;
    }
    ok();
    return align256(gh::refine_ws_bytes(g, n_cells));
}

int gh_refine(const gh_radar* radar, const gh_grid* grid, const void* d_y, const int64_t* d_cells, int32_t n_cells,
              int32_t max_iter, void* d_ws, size_t ws_bytes, double* d_theta, void* stream) {
    gh::Geom g;
    gh::GridP gp;
    int rc = make_geom(radar, g);
    if (rc || (rc = make_grid(grid, gp))) return rc;
    if (!d_y || !d_cells || !d_theta) return fail(GH_EINVAL, "NULL device pointer");
    if ((rc = check_aligned({d_y, d_cells, d_ws, d_theta}))) return rc;
    if (n_cells < 0 || n_cells > 65535) return fail(GH_EINVAL, "n_cells must be in [0, 65535]");
    if (max_iter < 1 || max_iter > 100) return fail(GH_EINVAL, "max_iter must be in [1, 100]");
    if (n_cells == 0) return ok();
    if (!d_ws) return fail(GH_EINVAL, "d_ws must be non-NULL");
    const size_t need = align256(gh::refine_ws_bytes(g, n_cells));
    if (ws_bytes < need) return fail(GH_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((rc = check_device())) return rc;
    hipError_t e = gh::launch_refine(g, gp, (const float2*)d_y, d_cells, n_cells, max_iter, d_ws, d_theta,
                                     (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gh_refine launch");
    return ok();
}

size_t gh_direct_points_workspace_bytes(const gh_radar* radar, int32_t n_points) {
    gh::Geom g;
    if (make_geom(radar, g)) return 0;
    if (n_points < 1 || n_points > 65535) {
        fail(GH_EINVAL, "n_points must be in [1, 65535]");
        return 0;
    }
    ok();
    return align256(gh::direct_points_ws_bytes(g, n_points));
}

int gh_direct_points(const gh_radar* radar, const void* d_y, const double* d_theta, int32_t n_points, double* d_value,
                     double* d_grad, double* d_grad_rx, void* d_ws, size_t ws_bytes, void* stream) {
    gh::Geom g;
    int rc = make_geom(radar, g);
    if (rc) return rc;
    if (n_points < 0 || n_points > 65535) return fail(GH_EINVAL, "n_points must be in [0, 65535]");
    if (!d_y || !d_theta || !d_value) return fail(GH_EINVAL, "d_y, d_theta and d_value must be non-NULL");
    if ((rc = check_aligned({d_y, d_theta, d_value, d_grad, d_grad_rx, d_ws}))) return rc;
    if (n_points == 0) return ok();
    if (!d_ws) return fail(GH_EINVAL, "d_ws must be non-NULL");
    const size_t need = align256(gh::direct_points_ws_bytes(g, n_points));
    if (ws_bytes < need) return fail(GH_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((rc = check_device())) return rc;
    hipError_t e = gh::launch_direct_points(g, (const float2*)d_y, d_theta, n_points, d_ws, d_value, d_grad,
                                            d_grad_rx, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gh_direct_points launch");
    return ok();
}

int gh_gh_points(const gh_radar* radar, const void* d_maps, int32_t map_dtype, int32_t interp, const double* d_theta,
                 int32_t n_points, double* d_value, double* d_grad, double* d_grad_rx, void* stream) {
    gh::Geom g;
    int rc = make_geom(radar, g);
    if (rc || (rc = check_map_dtype(g, map_dtype))) return rc;
    if (interp != GH_INTERP_BILINEAR && interp != GH_INTERP_BICUBIC)
        return fail(GH_EINVAL, "interp must be GH_INTERP_BILINEAR or GH_INTERP_BICUBIC");
    if (n_points < 0 || n_points > 65535) return fail(GH_EINVAL, "n_points must be in [0, 65535]");
    if (!d_maps || !d_theta || !d_value) return fail(GH_EINVAL, "d_maps, d_theta and d_value must be non-NULL");
    if ((rc = check_aligned({d_maps, d_theta, d_value, d_grad, d_grad_rx}))) return rc;
    if (n_points == 0) return ok();
    if ((rc = check_device())) return rc;
    hipError_t e = gh::launch_gh_points(g, d_maps, map_dtype, interp, d_theta, n_points, d_value, d_grad, d_grad_rx,
                                        (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gh_gh_points launch");
    return ok();
}

}  // extern "C"
