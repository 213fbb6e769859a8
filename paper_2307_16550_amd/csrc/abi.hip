// C ABI of the grid-hopping library: host-side validation, derived radar
// constants, workspace carving and dispatch to the gfx950 kernels.  Nothing is
// enqueued unless every argument has been checked; errors are reported as a
// gh_status plus a thread-local message, never as an exception.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <initializer_list>
#include <new>
#include <vector>

#include "gh_internal.h"

namespace {

thread_local char g_err[512] = "";
constexpr int kKnobs = 7;
thread_local int g_knob[kKnobs] = {};

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

// Host object of a batch of frames (include/gridhop.h).
struct gh_batch {
    int nf = 0, interp = 0, device = 0;
    int units[3] = {0, 0, 0};
    size_t lds1 = 0, lds2 = 0;   // LDS of the range and Doppler workgroups
    int nvx_t = 0, wave_f4 = 0;  // sweep column height, float4 per wave slice
    int waves = 4;
    int wg[3] = {0, 0, 0};
    int wg_max[3] = {0, 0, 0};
    int req_nch = 0, req_nrow = 0;   // requested map-pass tiles (0: each frame's planner)
    int loc_tile = 1;                // consecutive locations per sweep work unit
    long long points = 0;
    size_t ws_used = 0;
    gh::FrameDesc* d_table = nullptr;
    std::vector<gh::FrameDesc> table;   // host copy of the uploaded descriptors
};

namespace {

// Prefix the current error message with the frame's number.
int frame_fail(int rc, int f) {
    char msg[sizeof(g_err)];
    memcpy(msg, g_err, sizeof(msg));
    return fail(rc, "frame %d: %s", f, msg);
}

int current_device(int& dev) {
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "no usable HIP device");
    return GH_OK;
}

// Sizes of a batch's workspace: the table, then each frame's maps.
int batch_layout(const gh_frame* frames, int nf, std::vector<gh::Geom>& gs, std::vector<gh::GridP>& gps,
                 size_t& bytes) {
    if (!frames) return fail(GH_EINVAL, "frames is NULL");
    if (nf < 1 || nf > 65535) return fail(GH_EINVAL, "n_frames must be in [1, 65535]");
    gs.resize(nf);
    gps.resize(nf);
    bytes = align256((size_t)nf * sizeof(gh::FrameDesc));
    for (int f = 0; f < nf; ++f) {
        int rc = make_geom(&frames[f].radar, gs[f]);
        if (rc || (rc = make_grid(&frames[f].grid, gps[f]))) return frame_fail(rc, f);
        bytes += align256((size_t)gs[f].k * gs[f].nr * gs[f].nd * 8);
    }
    return GH_OK;
}

// Map-pass tiles and work units of every frame for the requested tiles (0:
// the frame's planner), the sweep's units for loc_tile locations each, and
// the largest LDS of each map pass.
int plan_units(std::vector<gh::FrameDesc>& table, int req_nch, int req_nrow, int loc_tile, int units_out[3],
               size_t& lds1, size_t& lds2) {
    long long units[3] = {0, 0, 0};
    lds1 = lds2 = 0;
    for (size_t f = 0; f < table.size(); ++f) {
        gh::FrameDesc& d = table[f];
        size_t l1, l2;
        gh::rd_maps_plan(d.g, d.nch, l1, d.nrow, d.pre_lds, l2);
        if (req_nch > 0 || req_nrow > 0) {
            if (req_nch > 0) d.nch = req_nch;
            if (req_nrow > 0) d.nrow = req_nrow;
            gh::rd_maps_shape(d.g, d.nch, d.nrow, l1, d.pre_lds, l2);
        }
        lds1 = l1 > lds1 ? l1 : lds1;
        lds2 = l2 > lds2 ? l2 : lds2;
        d.nunit[0] = d.g.k * d.g.pr * (d.g.mc / d.nch);
        d.nunit[1] = d.g.k * (d.g.nr / d.nrow);
        d.nunit[2] = (d.gp.nloc + loc_tile - 1) / loc_tile;
        for (int w = 0; w < 3; ++w) {
            d.unit0[w] = (int)units[w];
            units[w] += d.nunit[w];
        }
    }
    for (int w = 0; w < 3; ++w) {
        if (units[w] >= (1LL << 31)) return fail(GH_EUNSUPPORTED, "batch has more than 2^31 work units");
        units_out[w] = (int)units[w];
    }
    // the map passes of a batch also hold the current frame's descriptor in LDS
    if (lds1 + sizeof(gh::FrameDesc) > 65536 || lds2 + sizeof(gh::FrameDesc) > 65536)
        return fail(GH_EUNSUPPORTED, "map passes of this batch need more than 64 KB of LDS");
    return GH_OK;
}

int check_waves(int waves, int wave_f4) {
    if (waves != 1 && waves != 2 && waves != 4) return fail(GH_EINVAL, "sweep_waves must be 1, 2 or 4");
    if ((size_t)waves * wave_f4 * 16 > 65536)
        return fail(GH_EUNSUPPORTED, "%d sweep waves need %zu bytes of LDS (limit 65536)", waves,
                    (size_t)waves * wave_f4 * 16);
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
    size_t b = align256((size_t)gp.nloc * sizeof(gh_peak)) + align256(gh::bomp_fit_ws_bytes(g)) +
               align256(gh::bomp_atom_vec_bytes(g));
    if (use_direct)
        b += align256(gh::direct_ws_bytes(g, gp, gemm_dtype));
    else
        b += align256((size_t)g.k * g.nr * g.nd * sizeof(float2));   // maps of the residual
    return b + align256(gh::peak_split_ws_bytes());                   // the selection's split maximum
}

// Start of the split maximum's part of a Block-OMP workspace.
static char* bomp_split_ws(const gh::Geom& g, const gh::GridP& gp, int32_t use_direct, int32_t gemm_dtype, char* ws) {
    ws += align256((size_t)gp.nloc * sizeof(gh_peak)) + align256(gh::bomp_fit_ws_bytes(g)) +
          align256(gh::bomp_atom_vec_bytes(g));
    return ws + (use_direct ? align256(gh::direct_ws_bytes(g, gp, gemm_dtype))
                            : align256((size_t)g.k * g.nr * g.nd * sizeof(float2)));
}

// Shared checks of the Block-OMP entry points; sets g, gp.
static int bomp_common(const gh_radar* radar, const gh_grid* grid, int32_t use_direct, int32_t interp,
                       int32_t gemm_dtype, int32_t max_support, gh::Geom& g, gh::GridP& gp) {
    int rc = make_geom(radar, g);
    if (rc || (rc = make_grid(grid, gp)) || (rc = check_gemm(gemm_dtype))) return rc;
    if (use_direct != 0 && use_direct != 1) return fail(GH_EINVAL, "use_direct must be 0 or 1");
    if (!use_direct && (rc = check_sweep_limits(g, interp))) return rc;
    if (max_support < 1 || max_support > GH_MAX_SUPPORT)
        return fail(GH_EINVAL, "max_support must be in [1, %d]", GH_MAX_SUPPORT);
    return GH_OK;
}

// Decision on the residual (y itself at n_support == 0) and selection into
// support[n_support].  Grid hopping: the maps of y go to d_maps at
// n_support == 0; later, the maps of the residual are built in the workspace
// (the range rows the sweep reads) from them and the atom maps the previous
// fit left in the workspace, or by
// the FFT of the residual where the atoms' Doppler table does not fit (or
// with GH_BOMP_MAPS=fft, diagnostics).  The maximum over the grid is split
// over several workgroups, with a ticket counter in the workspace that each
// such launch leaves at zero; at n_support == 0 the Doppler pass of the maps
// (grid hopping) or a one-workgroup maximum (direct) zeroes it first.
// Arguments already checked.
static hipError_t bomp_select_launch(const gh::Geom& g, const gh::GridP& gp, const void* d_y, const void* d_resid,
                                     void* d_maps, int32_t use_direct, int32_t interp, int32_t gemm_dtype,
                                     int64_t* d_support, int32_t n_support, gh_peak* d_selected, char* ws,
                                     hipStream_t st) {
    const float2* src = (const float2*)(n_support == 0 ? d_y : d_resid);
    char* split_ws = bomp_split_ws(g, gp, use_direct, gemm_dtype, ws);
    gh_peak* block = (gh_peak*)ws;
    ws += align256((size_t)gp.nloc * sizeof(gh_peak));
    ws += align256(gh::bomp_fit_ws_bytes(g));
    const float2* atom_vec = (const float2*)ws;
    ws += align256(gh::bomp_atom_vec_bytes(g));
    hipError_t e;
    if (use_direct) {
        e = gh::launch_direct(g, gp, src, gemm_dtype, ws, nullptr, block, d_support, n_support, st);
    } else if (n_support == 0) {
        e = gh::launch_rd_maps(g, src, d_maps, GH_MAP_C64, st, (unsigned*)split_ws);
        if (e == hipSuccess)
            e = gh::launch_gh_sweep(g, gp, d_maps, GH_MAP_C64, interp, nullptr, block, d_support, n_support, st);
    } else {
        const bool fft_only = gh::knob(GH_KNOB_BOMP_MAPS_FFT) != 0;
        float2* rmaps = (float2*)ws;
        if (!fft_only && gh::bomp_resid_maps_ok(g, n_support))
            e = gh::launch_bomp_resid_maps(g, gp, (const float2*)d_maps, atom_vec, n_support, rmaps, st);
        else
            e = gh::launch_rd_maps(g, src, rmaps, GH_MAP_C64, st);
        if (e == hipSuccess)
            e = gh::launch_gh_sweep(g, gp, rmaps, GH_MAP_C64, interp, nullptr, block, d_support, n_support, st);
    }
    if (e != hipSuccess) return e;
    if (n_support == 0 && use_direct)
        return gh::launch_peak_final(block, gp.nloc, d_selected, d_support + n_support, st, (unsigned*)split_ws);
    return gh::launch_peak_final_split(block, gp.nloc, d_selected, d_support + n_support, split_ws, st);
}

static hipError_t bomp_fit_launch(const gh::Geom& g, const gh::GridP& gp, const void* d_y, void* d_resid,
                                  const int64_t* d_support, int32_t n_selected, void* d_alpha, char* ws,
                                  hipStream_t st) {
    char* fit_ws = ws + align256((size_t)gp.nloc * sizeof(gh_peak));
    float2* atom_vec = (float2*)(fit_ws + align256(gh::bomp_fit_ws_bytes(g)));
    return gh::launch_bomp_fit(g, gp, (const float2*)d_y, (float2*)d_resid, d_support, n_selected,
                               (float2*)d_alpha, fit_ws, atom_vec, st);
}

static int bomp_select_checks(const gh::GridP& gp, const void* d_y, const void* d_resid, const void* d_maps,
                              int32_t use_direct, const int64_t* d_support, int32_t n_support, int32_t max_support,
                              const gh_peak* d_selected, const void* d_ws) {
    if (!d_y || !d_support || !d_ws || (n_support > 0 && !d_resid)) return fail(GH_EINVAL, "NULL device pointer");
    if (!use_direct && !d_maps) return fail(GH_EINVAL, "d_maps must be non-NULL for grid hopping");
    if (int rc = check_aligned({d_y, d_resid, d_maps, d_support, d_selected, d_ws})) return rc;
    if (n_support < 0 || n_support >= max_support)
        return fail(GH_EINVAL, "n_support = %d must be in [0, max_support)", n_support);
    if (n_support + 1 > gp.nloc * (long long)gp.nv) return fail(GH_EINVAL, "support larger than the grid");
    return GH_OK;
}

int gh_bomp_step(const gh_radar* radar, const gh_grid* grid, const void* d_y, void* d_resid, void* d_maps,
                 int32_t use_direct, int32_t interp, int32_t gemm_dtype, int64_t* d_support, int32_t n_support,
                 int32_t max_support, void* d_alpha, gh_peak* d_selected, void* d_ws, size_t ws_bytes, void* stream) {
    gh::Geom g;
    gh::GridP gp;
    int rc = bomp_common(radar, grid, use_direct, interp, gemm_dtype, max_support, g, gp);
    if (rc) return rc;
    if (!d_resid || !d_alpha) return fail(GH_EINVAL, "NULL device pointer");
    if ((rc = bomp_select_checks(gp, d_y, d_resid, d_maps, use_direct, d_support, n_support, max_support, d_selected,
                                 d_ws)) ||
        (rc = check_aligned({d_alpha})))
        return rc;
    const size_t need = gh_bomp_workspace_bytes(radar, grid, use_direct, gemm_dtype);
    if (ws_bytes < need) return fail(GH_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((rc = check_device())) return rc;
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = bomp_select_launch(g, gp, d_y, d_resid, d_maps, use_direct, interp, gemm_dtype, d_support,
                                      n_support, d_selected, (char*)d_ws, st);
    if (e == hipSuccess) e = bomp_fit_launch(g, gp, d_y, d_resid, d_support, n_support + 1, d_alpha, (char*)d_ws, st);
    if (e != hipSuccess) return hip_fail(e, "gh_bomp_step launch");
    return ok();
}

int gh_bomp_select(const gh_radar* radar, const gh_grid* grid, const void* d_y, const void* d_resid, void* d_maps,
                   int32_t use_direct, int32_t interp, int32_t gemm_dtype, int64_t* d_support, int32_t n_support,
                   int32_t max_support, gh_peak* d_selected, void* d_ws, size_t ws_bytes, void* stream) {
    gh::Geom g;
    gh::GridP gp;
    int rc = bomp_common(radar, grid, use_direct, interp, gemm_dtype, max_support, g, gp);
    if (rc) return rc;
    if ((rc = bomp_select_checks(gp, d_y, d_resid, d_maps, use_direct, d_support, n_support, max_support, d_selected,
                                 d_ws)))
        return rc;
    const size_t need = gh_bomp_workspace_bytes(radar, grid, use_direct, gemm_dtype);
    if (ws_bytes < need) return fail(GH_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((rc = check_device())) return rc;
    const hipError_t e = bomp_select_launch(g, gp, d_y, d_resid, d_maps, use_direct, interp, gemm_dtype, d_support,
                                            n_support, d_selected, (char*)d_ws, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gh_bomp_select launch");
    return ok();
}

int gh_bomp_seed(const gh_radar* radar, const gh_grid* grid, int32_t interp, const gh_peak* d_block,
                 int64_t* d_support, int32_t max_support, gh_peak* d_selected, void* d_ws, size_t ws_bytes,
                 void* stream) {
    gh::Geom g;
    gh::GridP gp;
    int rc = bomp_common(radar, grid, 0, interp, GH_GEMM_F32, max_support, g, gp);
    if (rc) return rc;
    if (!d_block || !d_support || !d_ws) return fail(GH_EINVAL, "NULL device pointer");
    if ((rc = check_aligned({d_block, d_support, d_selected, d_ws}))) return rc;
    const size_t need = gh_bomp_workspace_bytes(radar, grid, 0, GH_GEMM_F32);
    if (ws_bytes < need) return fail(GH_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((rc = check_device())) return rc;
    char* split_ws = bomp_split_ws(g, gp, 0, GH_GEMM_F32, (char*)d_ws);
    // the grid maximum straight into the support and the selected peak, zeroing
    // the counter of the later selections' split maximum
    const hipError_t e = gh::launch_peak_final(d_block, gp.nloc, d_selected, d_support, (hipStream_t)stream,
                                               (unsigned*)split_ws);
    if (e != hipSuccess) return hip_fail(e, "gh_bomp_seed launch");
    return ok();
}

int gh_bomp_fit(const gh_radar* radar, const gh_grid* grid, const void* d_y, void* d_resid, const int64_t* d_support,
                int32_t n_selected, int32_t max_support, void* d_alpha, void* d_ws, size_t ws_bytes, void* stream) {
    gh::Geom g;
    gh::GridP gp;
    int rc = bomp_common(radar, grid, 0, GH_INTERP_BILINEAR, GH_GEMM_F32, max_support, g, gp);
    if (rc) return rc;
    if (!d_y || !d_resid || !d_support || !d_alpha || !d_ws) return fail(GH_EINVAL, "NULL device pointer");
    if ((rc = check_aligned({d_y, d_resid, d_support, d_alpha, d_ws}))) return rc;
    if (n_selected < 1 || n_selected > max_support)
        return fail(GH_EINVAL, "n_selected = %d must be in [1, max_support]", n_selected);
    if (n_selected > gp.nloc * (long long)gp.nv) return fail(GH_EINVAL, "support larger than the grid");
    // the part every Block-OMP workspace layout shares: block peaks, fit partials, atom maps
    const size_t need = align256((size_t)gp.nloc * sizeof(gh_peak)) + align256(gh::bomp_fit_ws_bytes(g)) +
                        align256(gh::bomp_atom_vec_bytes(g));
    if (ws_bytes < need) return fail(GH_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((rc = check_device())) return rc;
    const hipError_t e = bomp_fit_launch(g, gp, d_y, d_resid, d_support, n_selected, d_alpha, (char*)d_ws,
                                         (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gh_bomp_fit launch");
    return ok();
}

int gh_refine_noalloc(const gh_radar* radar, const gh_grid* grid, const void* d_y, const int64_t* d_cells,
                      int32_t n_cells, int32_t max_iter, double* d_theta, int32_t* d_status, void* stream) {
    gh::Geom g;
    gh::GridP gp;
    int rc = make_geom(radar, g);
    if (rc || (rc = make_grid(grid, gp))) return rc;
    if (!d_y || !d_cells || !d_theta) return fail(GH_EINVAL, "NULL device pointer");
    if ((rc = check_aligned({d_y, d_cells, d_theta, d_status}))) return rc;
    if (n_cells < 0) return fail(GH_EINVAL, "n_cells must be non-negative");
    if (n_cells > GH_REFINE_NOALLOC_MAX_CELLS)
        return fail(GH_EUNSUPPORTED, "gh_refine_noalloc takes at most %d cells (got %d); use gh_refine",
                    GH_REFINE_NOALLOC_MAX_CELLS, n_cells);
    if (max_iter < 1 || max_iter > 100) return fail(GH_EINVAL, "max_iter must be in [1, 100]");
    if (n_cells == 0) return ok();
    if ((rc = check_device())) return rc;
    hipError_t e = gh::launch_refine_noalloc(g, gp, (const float2*)d_y, d_cells, n_cells, max_iter, d_theta, d_status,
                                             (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gh_refine_noalloc launch");
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
              int32_t max_iter, void* d_ws, size_t ws_bytes, double* d_theta, int32_t* d_status, void* stream) {
    gh::Geom g;
    gh::GridP gp;
    int rc = make_geom(radar, g);
    if (rc || (rc = make_grid(grid, gp))) return rc;
    if (!d_y || !d_cells || !d_theta) return fail(GH_EINVAL, "NULL device pointer");
    if ((rc = check_aligned({d_y, d_cells, d_ws, d_theta, d_status}))) return rc;
    if (n_cells < 0 || n_cells > 65535) return fail(GH_EINVAL, "n_cells must be in [0, 65535]");
    if (max_iter < 1 || max_iter > 100) return fail(GH_EINVAL, "max_iter must be in [1, 100]");
    if (n_cells == 0) return ok();
    if (!d_ws) return fail(GH_EINVAL, "d_ws must be non-NULL");
    const size_t need = align256(gh::refine_ws_bytes(g, n_cells));
    if (ws_bytes < need) return fail(GH_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    if ((rc = check_device())) return rc;
    hipError_t e = gh::launch_refine(g, gp, (const float2*)d_y, d_cells, n_cells, max_iter, d_ws, d_theta,
                                     d_status, (hipStream_t)stream);
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

int gh_range_spectra(const gh_radar* radar, const void* d_y, void* d_spectra, void* stream) {
    gh::Geom g;
    int rc = make_geom(radar, g);
    if (rc) return rc;
    if (!d_y || !d_spectra) return fail(GH_EINVAL, "d_y and d_spectra must be non-NULL");
    if ((rc = check_aligned({d_y, d_spectra}))) return rc;
    const size_t ybytes = (size_t)g.k * g.mc * g.ms * 8, sbytes = (size_t)g.k * g.nr * g.mc * 8;
    const char *y0 = (const char*)d_y, *s0 = (const char*)d_spectra;
    if (y0 < s0 + sbytes && s0 < y0 + ybytes) return fail(GH_EINVAL, "d_y and d_spectra overlap");
    if ((rc = check_device())) return rc;
    hipError_t e = gh::launch_range_spectra(g, (const float2*)d_y, (float2*)d_spectra, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gh_range_spectra launch");
    return ok();
}

size_t gh_factored_workspace_bytes(const gh_radar* radar, const gh_grid* grid, int32_t method) {
    gh::Geom g;
    gh::GridP gp;
    if (make_geom(radar, g) || make_grid(grid, gp)) return 0;
    if (method != GH_FACTOR_DIRECT && method != GH_FACTOR_GRID_HOPPING) {
        fail(GH_EINVAL, "method must be GH_FACTOR_DIRECT or GH_FACTOR_GRID_HOPPING");
        return 0;
    }
    ok();
    return gh::factored_ws_bytes(g, gp, method);
}

int gh_factored_decision(const gh_radar* radar, const gh_grid* grid, int32_t method, int32_t range_interp,
                         int32_t gemm_dtype, const void* d_input, void* d_ws, size_t ws_bytes, float* d_loc,
                         float* d_vel, gh_peak* d_result, void* stream) {
    gh::Geom g;
    gh::GridP gp;
    int rc = make_geom(radar, g);
    if (rc || (rc = make_grid(grid, gp))) return rc;
    if (method != GH_FACTOR_DIRECT && method != GH_FACTOR_GRID_HOPPING)
        return fail(GH_EINVAL, "method must be GH_FACTOR_DIRECT or GH_FACTOR_GRID_HOPPING");
    if (method == GH_FACTOR_DIRECT && (rc = check_gemm(gemm_dtype))) return rc;
    if (method == GH_FACTOR_GRID_HOPPING && range_interp != GH_INTERP_BILINEAR && range_interp != GH_INTERP_BICUBIC &&
        range_interp != GH_INTERP_POLAR)
        return fail(GH_EINVAL, "range_interp must be GH_INTERP_BILINEAR, GH_INTERP_BICUBIC or GH_INTERP_POLAR");
    if (!d_input || !d_ws || !d_result) return fail(GH_EINVAL, "d_input, d_ws and d_result must be non-NULL");
    if ((rc = check_aligned({d_input, d_ws, d_loc, d_vel, d_result}))) return rc;
    const size_t need = gh::factored_ws_bytes(g, gp, method);
    if (ws_bytes < need) return fail(GH_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    // polar rule: circle angle per bin from the chord lengths of three neighbouring
    // range atoms, |f(a) - f(b)|^2 = 2 Ms - 2 Re <f(a), f(b)>
    double theta = 0.0;
    if (method == GH_FACTOR_GRID_HOPPING && range_interp == GH_INTERP_POLAR) {
        const double c = g.centered ? (g.ms - 1) / 2.0 : 0.0;
        double re1 = 0.0, re2 = 0.0;
        for (int s = 0; s < g.ms; ++s) {
            re1 += cos(2.0 * M_PI * (s - c) / g.nr);
            re2 += cos(4.0 * M_PI * (s - c) / g.nr);
        }
        theta = acos((g.ms - re2) / (2.0 * (g.ms - re1)) - 1.0);
    }
    if ((rc = check_device())) return rc;
    hipError_t e = gh::launch_factored(g, gp, method, range_interp, theta, gemm_dtype, d_input, d_ws, d_loc, d_vel,
                                       d_result, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "gh_factored_decision launch");
    return ok();
}

size_t gh_batch_workspace_bytes(const gh_frame* frames, int32_t n_frames) {
    std::vector<gh::Geom> gs;
    std::vector<gh::GridP> gps;
    size_t bytes = 0;
    if (batch_layout(frames, n_frames, gs, gps, bytes)) return 0;
    ok();
    return bytes;
}

int gh_batch_create(const gh_frame* frames, int32_t n_frames, int32_t interp, void* d_ws, size_t ws_bytes,
                    gh_batch** batch, void* stream) {
    if (!batch) return fail(GH_EINVAL, "batch is NULL");
    *batch = nullptr;
    std::vector<gh::Geom> gs;
    std::vector<gh::GridP> gps;
    size_t need = 0;
    int rc = batch_layout(frames, n_frames, gs, gps, need);
    if (rc) return rc;
    if (interp != GH_INTERP_BILINEAR && interp != GH_INTERP_BICUBIC)
        return fail(GH_EINVAL, "interp must be GH_INTERP_BILINEAR or GH_INTERP_BICUBIC");
    if (!d_ws) return fail(GH_EINVAL, "d_ws is NULL");
    if ((rc = check_aligned({d_ws}))) return rc;
    if (ws_bytes < need) return fail(GH_EWORKSPACE, "workspace of %zu bytes, %zu needed", ws_bytes, need);
    int nd_max = 0, chunk_max = 0;
    long long points = 0;
    std::vector<gh::FrameDesc> table(n_frames);
    char* maps = (char*)d_ws + align256((size_t)n_frames * sizeof(gh::FrameDesc));
    size_t lds1 = 0, lds2 = 0;
    for (int f = 0; f < n_frames; ++f) {
        const gh_frame& fr = frames[f];
        const gh::Geom& g = gs[f];
        const gh::GridP& gp = gps[f];
        if (!fr.d_y || !fr.d_block) return fail(GH_EINVAL, "frame %d: d_y and d_block must be non-NULL", f);
        if ((rc = check_aligned({fr.d_y, fr.d_decision, fr.d_block}))) return frame_fail(rc, f);
        if (g.nd < 16) return fail(GH_EUNSUPPORTED, "frame %d: N_d = %d < 16", f, g.nd);
        const int nvy = gp.n[3];
        if (nvy > 64) return fail(GH_EUNSUPPORTED, "frame %d: Nvy = %d > 64", f, nvy);
        const int parts = 64 / nvy;
        const int chunk = (gp.n[2] + parts - 1) / parts;
        if (chunk > 32) return fail(GH_EUNSUPPORTED, "frame %d: %d vx points per lane (limit 32)", f, chunk);
        gh::FrameDesc& d = table[f];
        memset(&d, 0, sizeof(d));
        d.g = g;
        d.gp = gp;
        d.y = (const float2*)fr.d_y;
        d.maps = maps;
        d.dec = fr.d_decision;
        d.block = fr.d_block;
        d.nvy = nvy;
        d.parts = parts;
        d.chunk = chunk;
        nd_max = g.nd > nd_max ? g.nd : nd_max;
        chunk_max = chunk > chunk_max ? chunk : chunk_max;
        points += (long long)gp.nloc * gp.nv;
        maps += align256((size_t)g.k * g.nr * g.nd * 8);
    }
    int nunits[3];
    if ((rc = plan_units(table, 0, 0, 1, nunits, lds1, lds2))) return rc;
    const int wave_f4 = gh::sweep_batch_slice_f4(interp, nd_max);
    int nvx_t = 0;
    gh::sweep_batch_nvx(chunk_max, nvx_t);
    int waves = 4;
    while (waves > 1 && (size_t)waves * wave_f4 * 16 > 65536) waves >>= 1;
    int device = 0;
    if ((rc = check_waves(waves, wave_f4)) || (rc = current_device(device))) return rc;
    gh_batch* b = new (std::nothrow) gh_batch;
    if (!b) return fail(GH_EINVAL, "out of host memory");
    b->device = device;
    b->nf = n_frames;
    b->interp = interp;
    for (int w = 0; w < 3; ++w) b->units[w] = nunits[w];
    b->lds1 = lds1;
    b->lds2 = lds2;
    b->nvx_t = nvx_t;
    b->wave_f4 = wave_f4;
    b->waves = waves;
    b->points = points;
    b->ws_used = need;
    b->wg_max[0] = gh::range_batch_max_workgroups(lds1);
    b->wg_max[1] = gh::doppler_batch_max_workgroups(lds2);
    b->wg_max[2] = gh::sweep_batch_max_workgroups(interp, nvx_t, waves, (size_t)waves * wave_f4 * 16);
    for (int w = 0; w < 3; ++w) {
        if (b->wg_max[w] < 1) {
            delete b;
            return fail(GH_EHIP, "occupancy query of the batch kernels failed");
        }
        b->wg[w] = b->wg_max[w];
    }
    b->d_table = (gh::FrameDesc*)d_ws;
    b->table.swap(table);
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(b->d_table, b->table.data(), b->table.size() * sizeof(gh::FrameDesc),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "gh_batch_create upload");
    }
    *batch = b;
    return ok();
}

int gh_batch_tune(gh_batch* batch, int32_t range_workgroups, int32_t doppler_workgroups, int32_t sweep_workgroups,
                  int32_t sweep_waves) {
    if (!batch) return fail(GH_EINVAL, "batch is NULL");
    const int req[3] = {range_workgroups, doppler_workgroups, sweep_workgroups};
    for (int w = 0; w < 3; ++w)
        if (req[w] < 0) return fail(GH_EINVAL, "workgroup counts must be >= 0");
    int rc;
    if (sweep_waves != 0 && (rc = check_waves(sweep_waves, batch->wave_f4))) return rc;
    if (sweep_waves != 0 && sweep_waves != batch->waves) {
        const int mx = gh::sweep_batch_max_workgroups(batch->interp, batch->nvx_t, sweep_waves,
                                                      (size_t)sweep_waves * batch->wave_f4 * 16);
        if (mx < 1) return fail(GH_EHIP, "occupancy query of the sweep failed");
        batch->waves = sweep_waves;
        batch->wg_max[2] = mx;
        if (sweep_workgroups == 0) batch->wg[2] = mx;
    }
    for (int w = 0; w < 3; ++w)
        if (req[w] > 0) batch->wg[w] = req[w];
    return ok();
}

int gh_batch_tune_tiles(gh_batch* batch, int32_t range_chirps, int32_t doppler_rows, int32_t sweep_locations,
                        void* stream) {
    if (!batch) return fail(GH_EINVAL, "batch is NULL");
    auto pow2_or_zero = [](int v) { return v == 0 || (v > 0 && v <= 4096 && (v & (v - 1)) == 0); };
    if (!pow2_or_zero(range_chirps) || !pow2_or_zero(doppler_rows))
        return fail(GH_EINVAL, "range_chirps and doppler_rows must be 0 or powers of two up to 4096");
    if (sweep_locations < 0 || sweep_locations > 64)
        return fail(GH_EINVAL, "sweep_locations must be in [0, 64]");
    int dev = -1;
    int rc = current_device(dev);
    if (rc) return rc;
    if (dev != batch->device) return fail(GH_EINVAL, "batch created on device %d, current device %d", batch->device, dev);
    std::vector<gh::FrameDesc> table = batch->table;
    const int loc_tile = sweep_locations > 0 ? sweep_locations : batch->loc_tile;
    int units[3];
    size_t lds1, lds2;
    if ((rc = plan_units(table, range_chirps, doppler_rows, loc_tile, units, lds1, lds2))) return rc;
    const int mx0 = gh::range_batch_max_workgroups(lds1), mx1 = gh::doppler_batch_max_workgroups(lds2);
    if (mx0 < 1 || mx1 < 1) return fail(GH_EHIP, "occupancy query of the map passes failed");
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(batch->d_table, table.data(), table.size() * sizeof(gh::FrameDesc),
                                  hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(e, "gh_batch_tune_tiles upload");
    batch->table.swap(table);
    for (int w = 0; w < 3; ++w) batch->units[w] = units[w];
    batch->lds1 = lds1;
    batch->lds2 = lds2;
    batch->wg_max[0] = batch->wg[0] = mx0;
    batch->wg_max[1] = batch->wg[1] = mx1;
    batch->req_nch = range_chirps;
    batch->req_nrow = doppler_rows;
    batch->loc_tile = loc_tile;
    return ok();
}

int gh_batch_get_info(const gh_batch* batch, gh_batch_info* info) {
    if (!batch || !info) return fail(GH_EINVAL, "batch and info must be non-NULL");
    memset(info, 0, sizeof(*info));
    info->n_frames = batch->nf;
    info->interp = batch->interp;
    for (int w = 0; w < 3; ++w) {
        info->units[w] = batch->units[w];
        info->workgroups[w] = batch->wg[w];
        info->max_workgroups[w] = batch->wg_max[w];
    }
    info->sweep_waves = batch->waves;
    info->column_height = batch->nvx_t;
    info->sweep_locations = batch->loc_tile;
    info->range_chirps = batch->req_nch;
    info->doppler_rows = batch->req_nrow;
    info->points = batch->points;
    info->workspace_bytes = (int64_t)batch->ws_used;
    return ok();
}

int gh_batch_run(const gh_batch* batch, gh_peak* d_argmax, void* stream) {
    if (!batch) return fail(GH_EINVAL, "batch is NULL");
    int dev = -1;
    int rc = check_aligned({d_argmax});
    if (rc || (rc = current_device(dev))) return rc;
    if (dev != batch->device) return fail(GH_EINVAL, "batch created on device %d, current device %d", batch->device, dev);
    hipStream_t st = (hipStream_t)stream;
    const gh::FrameDesc* t = batch->d_table;
    hipError_t e = gh::launch_rd_maps_batch(t, batch->nf, batch->units[0], batch->units[1], batch->lds1, batch->lds2,
                                            batch->wg[0], batch->wg[1], st);
    if (e == hipSuccess)
        e = gh::launch_sweep_batch(t, batch->nf, batch->units[2], batch->interp, batch->nvx_t, batch->wave_f4,
                                   batch->waves, batch->wg[2], batch->loc_tile, st);
    if (e == hipSuccess && d_argmax) e = gh::launch_peak_batch(t, batch->nf, d_argmax, st);
    if (e != hipSuccess) return hip_fail(e, "gh_batch_run launch");
    return ok();
}

int gh_batch_frame_maps(const gh_batch* batch, int32_t frame, void** d_maps) {
    if (!batch || !d_maps) return fail(GH_EINVAL, "batch and d_maps must be non-NULL");
    if (frame < 0 || frame >= batch->nf) return fail(GH_EINVAL, "frame %d outside [0, %d)", frame, batch->nf);
    *d_maps = batch->table[frame].maps;
    return ok();
}

void gh_batch_destroy(gh_batch* batch) { delete batch; }

}  // extern "C"

namespace gh {
int knob(int which) { return (which > 0 && which < kKnobs) ? g_knob[which] : 0; }
}  // namespace gh

extern "C" int gh_test_set_knob(int32_t knob, int32_t value) {
    int lo = 0, hi = 1;
    switch (knob) {
        case GH_KNOB_SWEEP_GENERIC: case GH_KNOB_BOMP_MAPS_FFT: case GH_KNOB_REFINE_SINGLE: break;
        case GH_KNOB_SWEEP_LDS_KIB: hi = 160; break;
        case GH_KNOB_REFINE_ROWS: hi = 4096; break;
        case GH_KNOB_REFINE_SPIN_LIMIT: hi = 1 << 30; break;
        default: return fail(GH_EINVAL, "unknown switch %d", knob);
    }
    if (value < lo || value > hi) return fail(GH_EINVAL, "switch %d: value %d outside [%d, %d]", knob, value, lo, hi);
    if (knob == GH_KNOB_SWEEP_LDS_KIB && value != 0 && value < 8)
        return fail(GH_EINVAL, "switch %d: LDS budget below 8 KiB", knob);
    if (knob == GH_KNOB_REFINE_ROWS && value != 0 && !pow2(value))
        return fail(GH_EINVAL, "switch %d: rows per workgroup must be a power of two", knob);
    const int prev = g_knob[knob];
    g_knob[knob] = value;
    ok();
    return prev;
}
