// Internal declarations of the gfx950 grid-hopping library: kernel parameter
// blocks (passed by value), device helpers and the host launchers that the
// C ABI layer (abi.hip) dispatches to.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gridhop.h"
#include "gridhop_test.h"

namespace gh {

// Per-thread override of a test switch (gridhop_test.h); 0 = default.
int knob(int which);

constexpr int kMaxRx = GH_MAX_RX;
constexpr int kMaxSupport = GH_MAX_SUPPORT;

// Radar constants in the form the kernels use.  Sensing functions (paper
// Sec. II, eqs. (1)-(2)) with the FMCW scaling: continuous map coordinates
// t_r = kr * R (range bins) and t_d = kd * U (Doppler bins); f_r = fr_per_m * R
// cycles per sample and f_d = fd_per_mps * U cycles per chirp.
struct Geom {
    double tx[2];
    double rx[kMaxRx][2];
    double kr;          // B * P_r / c
    double kd;          // f0 * Tc * P_d * Mc / c
    double fr_per_m;    // B / (c * Ms)
    double fd_per_mps;  // f0 * Tc / c
    int k, ms, mc, nr, nd, pr, pd;
    int log2_ms, log2_mc, log2_nr, log2_nd;
    int centered;
    float sign_r, sign_d;  // factor per period of the (centred) correlation: (-1)^(M-1) or 1
};

struct GridP {
    double lo[4];
    double step[4];
    int n[4];
    int nloc;   // n[0] * n[1]
    int nv;     // n[2] * n[3]
};

// ---- small device helpers -------------------------------------------------

// A pointer read from memory (a descriptor table) carries no address space, so
// its accesses compile to flat instructions; this marks it as global memory
// (all device arrays of the library are) so they compile to global ones.
// (Through an integer: a direct cast pair is folded away before address
// spaces are inferred.)
template <typename T>
__device__ __forceinline__ T* as_global(T* p) {
    return (T*)(__attribute__((address_space(1))) T*)(uintptr_t)p;
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// exp(-j 2 pi u) for a phase u = ph * 2^-32 cycles held in 32-bit fixed point
// (the wrap modulo one cycle is exact integer overflow).
__device__ __forceinline__ float2 expm_fixed(uint32_t ph) {
    float s, c;
    // sin/cos of pi * x with x = 2 * ph * 2^-32 in [0, 2)
    sincospif(__uint2float_rn(ph) * 4.656612873077393e-10f, &s, &c);
    return make_float2(c, -s);
}

// Round a phase in cycles (any sign or size) to 32-bit fixed point, modulo 1 cycle.
__host__ __device__ __forceinline__ uint32_t cycles_to_fixed(double cyc) {
    double f = cyc - floor(cyc);                   // [0, 1)
    double scaled = f * 4294967296.0;
    unsigned long long r = (unsigned long long)(scaled + 0.5);
    return (uint32_t)(r & 0xffffffffull);
}

// Round a phase in cycles to 64-bit fixed point (53 significant bits), modulo
// 1 cycle: the phase of sample n is then (fixed * n) mod 2^64, exact.
__host__ __device__ __forceinline__ uint64_t cycles_to_fixed64(double cyc) {
    const double f = cyc - floor(cyc);                       // [0, 1]
    const unsigned long long r = (unsigned long long)(f * 9007199254740992.0 + 0.5);   // 2^53
    return (uint64_t)(r & ((1ull << 53) - 1)) << 11;
}

// exp(-j 2 pi ph / 2^64) in FP64.
__device__ __forceinline__ double2 expm_fixed64(uint64_t ph) {
    double s, c;
    // sin/cos of pi * x with x = 2 * ph * 2^-64 in [0, 2), from the top 53 bits
    sincospi((double)(ph >> 11) * 2.220446049250313e-16, &s, &c);
    return make_double2(c, -s);
}

// Signed increment in cycles to a 32-bit two's complement fixed-point step.
__host__ __device__ __forceinline__ uint32_t cycles_to_fixed_step(double cyc) {
    return cycles_to_fixed(cyc);  // modular arithmetic: the step is also taken mod 1 cycle
}

// ---- map storage (gh_map_dtype) ---------------------------------------------
// Bytes per complex map value: 8 (complex64) or 4 (a pair of 16-bit floats).
__host__ __device__ constexpr int map_elem_bytes(int dt) { return dt == GH_MAP_C64 ? 8 : 4; }

__device__ __forceinline__ float half_bits_to_float(uint32_t bits, int dt) {
    if (dt == GH_MAP_BF16) return __uint_as_float(bits << 16);
    return (float)__builtin_bit_cast(_Float16, (unsigned short)bits);
}

__device__ __forceinline__ uint32_t float_to_half_bits(float v, int dt) {
    if (dt == GH_MAP_BF16) return (uint32_t)__builtin_bit_cast(unsigned short, (__bf16)v);
    return (uint32_t)__builtin_bit_cast(unsigned short, (_Float16)v);
}

// One complex map value at byte offset `off`.
template <int DT>
__device__ __forceinline__ float2 map_ld1(const char* base, uint32_t off) {
    if constexpr (DT == GH_MAP_C64) {
        return *reinterpret_cast<const float2*>(base + off);
    } else {
        const uint32_t u = *reinterpret_cast<const uint32_t*>(base + off);
        return make_float2(half_bits_to_float(u & 0xffffu, DT), half_bits_to_float(u >> 16, DT));
    }
}

// Two consecutive complex map values at byte offset `off` as (re0, im0, re1, im1).
template <int DT>
__device__ __forceinline__ float4 map_ld2(const char* base, uint32_t off) {
    if constexpr (DT == GH_MAP_C64) {
        return *reinterpret_cast<const float4*>(base + off);
    } else {
        const uint2 u = *reinterpret_cast<const uint2*>(base + off);
        return make_float4(half_bits_to_float(u.x & 0xffffu, DT), half_bits_to_float(u.x >> 16, DT),
                           half_bits_to_float(u.y & 0xffffu, DT), half_bits_to_float(u.y >> 16, DT));
    }
}

// Scale of the stored maps: the half formats hold Z / (Ms * Mc).
__host__ __device__ __forceinline__ float map_scale(int ms, int mc, int dt) {
    return dt == GH_MAP_C64 ? 1.f : (float)ms * (float)mc;
}

// 1 / sqrt(v) in FP64 for v >= 0: the hardware estimate refined by two Newton
// steps (relative error at the level of FP64 rounding); 0 for v == 0, which
// makes the unit vector of a zero-length leg zero.
__device__ __forceinline__ double rsqrt_fp64(double v) {
    if (!(v > 0.0)) return 0.0;
    const double h = 0.5 * v;
    double y = __builtin_amdgcn_rsq(v);
    y = y * fma(-h * y, y, 1.5);
    y = y * fma(-h * y, y, 1.5);
    return y;
}

// Bistatic geometry of one location and receiver, FP64.
__device__ __forceinline__ void bistatic(const Geom& g, int q, double x, double y, double& r, double& wx,
                                         double& wy) {
    double dx0 = x - g.tx[0], dy0 = y - g.tx[1];
    double dx1 = x - g.rx[q][0], dy1 = y - g.rx[q][1];
    double n0 = sqrt(dx0 * dx0 + dy0 * dy0);
    double n1 = sqrt(dx1 * dx1 + dy1 * dy1);
    r = n0 + n1;
    wx = 0.0;
    wy = 0.0;
    if (n0 > 0.0) { wx += dx0 / n0; wy += dy0 / n0; }
    if (n1 > 0.0) { wx += dx1 / n1; wy += dy1 / n1; }
}

// (value, index) max with ties to the lowest index.
__device__ __forceinline__ void peak_merge(float& v, int& i, float v2, int i2) {
    if (v2 > v || (v2 == v && i2 < i)) { v = v2; i = i2; }
}

__device__ __forceinline__ void wave_peak(float& v, int& i) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        float v2 = __shfl_xor(v, off, 64);
        int i2 = __shfl_xor(i, off, 64);
        peak_merge(v, i, v2, i2);
    }
}

// The same maximum on the VALU alone (no LDS round trips, which queue behind
// a sweep's table traffic): within each row of 16 lanes, merges with the row
// rotated by 1, 2, 4 and 8 lanes (DPP row_ror), then the four row results by
// lane reads.  Every lane ends with the wave's maximum.  All 64 lanes must be
// active.
template <int CTRL>
__device__ __forceinline__ void peak_merge_dpp(float& v, int& i) {
    const float v2 = __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
    const int i2 = __builtin_amdgcn_update_dpp(0, i, CTRL, 0xf, 0xf, false);
    peak_merge(v, i, v2, i2);
}

__device__ __forceinline__ void wave_peak_rows(float& v, int& i) {
    peak_merge_dpp<0x121>(v, i);   // row_ror:1
    peak_merge_dpp<0x122>(v, i);   // row_ror:2
    peak_merge_dpp<0x124>(v, i);   // row_ror:4
    peak_merge_dpp<0x128>(v, i);   // row_ror:8
    float rv = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 0));
    int ri = __builtin_amdgcn_readlane(i, 0);
#pragma unroll
    for (int r = 1; r < 4; ++r)
        peak_merge(rv, ri, __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 16 * r)),
                   __builtin_amdgcn_readlane(i, 16 * r));
    v = rv;
    i = ri;
}

// Per-location epilogue shared by the decision kernels: write the slab (if
// `dec`), reduce its maximum (ties -> lowest index) skipping excluded cells,
// and store the block peak.  `acc[j]` holds the value of point tid + j*NT.
template <int NT, int NPTS>
__device__ __forceinline__ void slab_epilogue(const float (&acc)[NPTS], int nv, int loc, float* __restrict__ dec,
                                              gh_peak* __restrict__ block, const int* excl_local, int nex,
                                              float* red_v, int* red_i) {
    const int tid = threadIdx.x;
    float best_v = -INFINITY;
    int best_i = 0x7fffffff;
#pragma unroll
    for (int j = 0; j < NPTS; ++j) {
        const int v = tid + j * NT;
        if (v < nv) {
            if (dec) dec[(size_t)loc * nv + v] = acc[j];
            bool skip = false;
            for (int e = 0; e < nex; ++e) skip |= (excl_local[e] == v);
            if (!skip) peak_merge(best_v, best_i, acc[j], v);
        }
    }
    wave_peak(best_v, best_i);
    const int wid = tid >> 6;
    if ((tid & 63) == 0) {
        red_v[wid] = best_v;
        red_i[wid] = best_i;
    }
    __syncthreads();
    if (tid == 0) {
        for (int w = 1; w < NT / 64; ++w) peak_merge(best_v, best_i, red_v[w], red_i[w]);
        gh_peak p;
        p.value = best_v;
        p.reserved = 0;
        p.index = (int64_t)loc * nv + (best_i == 0x7fffffff ? 0 : best_i);
        block[loc] = p;
    }
}

// Largest of n block maxima (ties to the lowest index), reduced by a whole
// workgroup of up to 1024 threads; the result is valid in thread 0.  red_v and
// red_i are LDS arrays of blockDim.x / 64 entries.
// Maximum (ties to the lowest index) of n block peaks by the whole workgroup
// (every lane active); the result is in thread 0.  Linear grid indices fit in
// 32 bits (grids have fewer than 2^31 points), so the merges across lanes are
// the VALU-only wave_peak_rows: per wave, then over the waves' results by wave 0.
__device__ __forceinline__ void reduce_block_peaks(const gh_peak* __restrict__ blk, int n, float& bv, long long& bi,
                                                   float* red_v, long long* red_i) {
    bv = -INFINITY;
    int b32 = 0x7fffffff;
    // sixteen independent loads in flight per thread, then their comparisons
    for (int b0 = threadIdx.x; b0 < n; b0 += 16 * blockDim.x) {
        gh_peak p[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int b = b0 + k * (int)blockDim.x;
            if (b < n) p[k] = blk[b];
        }
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const int b = b0 + k * (int)blockDim.x;
            if (b < n) peak_merge(bv, b32, p[k].value, (int)p[k].index);
        }
    }
    wave_peak_rows(bv, b32);
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 0) {
        red_v[wid] = bv;
        red_i[wid] = b32;
    }
    __syncthreads();
    if (wid == 0) {
        const int nw = (int)(blockDim.x >> 6);
        bv = lane < nw ? red_v[lane] : -INFINITY;
        b32 = lane < nw ? (int)red_i[lane] : 0x7fffffff;
        wave_peak_rows(bv, b32);
    }
    bi = b32;
}

// Exclusion list entries that fall in this location's slab (thread 0 only).
__device__ __forceinline__ int local_exclusions(const int64_t* excl, int nexcl, int loc, int nv, int* out) {
    int n = 0;
    const int64_t base = (int64_t)loc * nv;
    for (int e = 0; e < nexcl; ++e) {
        const int64_t d = excl[e] - base;
        if (d >= 0 && d < nv) out[n++] = (int)d;
    }
    return n;
}

// ---- batches of frames --------------------------------------------------------
// One frame of a batch, in a device-resident table.  The persistent batch
// kernels walk a global sequence of work units in which each frame's units are
// contiguous: range units (q, p, chirp group), Doppler units (q, row group),
// sweep units (one location each, one wave per unit).
struct FrameDesc {
    Geom g;
    GridP gp;
    const float2* y;     // complex64 [K][Mc][Ms]
    char* maps;          // complex64 [K][N_r][N_d] (batch workspace)
    float* dec;          // decision volume or NULL
    gh_peak* block;      // [Nx*Ny] block maxima
    int unit0[3];        // first unit of the frame: range, Doppler, sweep
    int nunit[3];        // units of the frame
    int nch, nrow, pre_lds;   // map pass shapes (rd_maps_plan)
    int nvy, parts, chunk;    // sweep columns: lane = part * nvy + ivy, part < parts owns vx rows [part*chunk, +chunk)
};

// ---- host launchers (return hipError_t of the launches) --------------------

// clear: optional counter zeroed by the Doppler pass (see launch_peak_final_split).
hipError_t launch_rd_maps(const Geom& g, const float2* y, void* maps, int map_dtype, hipStream_t st,
                          unsigned* clear = nullptr);

// Work decomposition of the map passes: nch chirps per range workgroup (LDS
// lds1), nrow range rows per Doppler workgroup (LDS lds2, pre-twiddles in LDS
// when pre_lds).
void rd_maps_plan(const Geom& g, int& nch, size_t& lds1, int& nrow, int& pre_lds, size_t& lds2);
// The same for a requested nch and nrow (powers of two), clamped in place.
void rd_maps_shape(const Geom& g, int& nch, int& nrow, size_t& lds1, int& pre_lds, size_t& lds2);

// Batch launches (frames: device table of nf descriptors).  Workgroup counts
// are the persistent grid sizes; each launch clamps them to its unit count.
hipError_t launch_rd_maps_batch(const FrameDesc* frames, int nf, int range_units, int doppler_units, size_t lds1,
                                size_t lds2, int wg_range, int wg_doppler, hipStream_t st);
// Sweep: `waves` waves per workgroup, each with a private LDS slice of
// wave_f4 float4 (FastGeo records of up to GH_MAX_RX receivers, then the
// Doppler table of the largest N_d); nvx_t is the compile-time column height.
int sweep_batch_slice_f4(int interp, int nd_max);
bool sweep_batch_nvx(int chunk_max, int& nvx_t);
int sweep_batch_max_workgroups(int interp, int nvx_t, int waves, size_t lds);
hipError_t launch_sweep_batch(const FrameDesc* frames, int nf, int units, int interp, int nvx_t, int wave_f4,
                              int waves, int workgroups, int loc_tile, hipStream_t st);
hipError_t launch_peak_batch(const FrameDesc* frames, int nf, gh_peak* argmax, hipStream_t st);
int range_batch_max_workgroups(size_t lds);
int doppler_batch_max_workgroups(size_t lds);

// The range pass alone into compact per-chirp spectra, complex64 [K][N_r][Mc].
hipError_t launch_range_spectra(const Geom& g, const float2* y, float2* spectra, hipStream_t st);

// Factorised decisions (eqs. (5)-(6)): see factor.hip.
size_t factored_ws_bytes(const Geom& g, const GridP& gp, int method);
hipError_t launch_factored(const Geom& g, const GridP& gp, int method, int range_interp, double polar_theta,
                           int gemm, const void* input, void* ws, float* loc, float* vel, gh_peak* result,
                           hipStream_t st);
// The range zoom of the direct decision alone: G_q[x][m], float2 [K][Nloc][Mc].
hipError_t launch_direct_range(const Geom& g, const GridP& gp, const float2* y, int gemm, float2* G, hipStream_t st);

hipError_t launch_gh_sweep(const Geom& g, const GridP& gp, const void* maps, int map_dtype, int interp, float* dec,
                           gh_peak* block, const int64_t* excl, int nexcl, hipStream_t st);

// Column variant of the sweep (power-of-two vy slabs); plan() returns false
// when the shape needs the generic kernel.
bool sweep_columns_plan(const Geom& g, const GridP& gp, int interp, int& lpb, int& log2nvy, size_t& lds);
hipError_t launch_gh_sweep_columns(const Geom& g, const GridP& gp, int lpb, int log2nvy, size_t lds,
                                   const void* maps, int map_dtype, int interp, float* dec, gh_peak* block,
                                   const int64_t* excl, int nexcl, hipStream_t st);

// Global maximum of nblock block maxima (one workgroup); also zeroes *clear
// when it is not null.
hipError_t launch_peak_final(const gh_peak* block, int nblock, gh_peak* out, int64_t* support_slot,
                             hipStream_t st, unsigned* clear = nullptr);
// The same maximum split over several workgroups, the last of which merges
// their shares.  ws: peak_split_ws_bytes() of device memory whose first word
// (a ticket counter) is zero; the launch leaves it zero.
size_t peak_split_ws_bytes();
hipError_t launch_peak_final_split(const gh_peak* block, int nblock, gh_peak* out, int64_t* support_slot, void* ws,
                                   hipStream_t st);

size_t direct_ws_bytes(const Geom& g, const GridP& gp, int gemm);
hipError_t launch_direct(const Geom& g, const GridP& gp, const float2* y, int gemm, void* ws, float* dec,
                         gh_peak* block, const int64_t* excl, int nexcl, hipStream_t st);

size_t bomp_fit_ws_bytes(const Geom& g);
// The fit also writes, per receiver and fitted atom, the atom's maps as an
// outer product alpha_t R_t[i] D_t[l] (closed-form Dirichlet sums along range
// and Doppler): atom_vec [K][GH_MAX_SUPPORT][N_r + N_d] complex64.
size_t bomp_atom_vec_bytes(const Geom& g);
hipError_t launch_bomp_fit(const Geom& g, const GridP& gp, const float2* y, float2* resid,
                           const int64_t* support, int nsel, float2* alpha, void* ws, float2* atom_vec,
                           hipStream_t st);
// Maps of the residual Y - sum_t alpha_t A(theta_t) from the maps of Y by
// linearity, with the atom vectors of the last fit.  Applies while nsel * N_d
// fits the kernel's table (bomp_resid_maps_ok).  Only the range rows that a
// sweep over the grid gp can read (a bound from its bistatic range span) are
// written; the other rows of `out` keep their contents.
bool bomp_resid_maps_ok(const Geom& g, int nsel);
// support[0] (and *selected, if given) from *argmax; *counter zeroed.
hipError_t launch_bomp_resid_maps(const Geom& g, const GridP& gp, const float2* maps_y, const float2* atom_vec,
                                  int nsel, float2* out, hipStream_t st);

size_t refine_ws_bytes(const Geom& g, int ncells);
// status (nullable): int32, set to the number of cells whose estimate is NaN
// (a cluster barrier wait expired).
hipError_t launch_refine(const Geom& g, const GridP& gp, const float2* y, const int64_t* cells, int ncells,
                         int max_iter, void* ws, double* theta, int* status, hipStream_t st);
// The same with the library's own static scratch (gh_refine_noalloc): no
// allocation; ncells <= GH_REFINE_NOALLOC_MAX_CELLS.
hipError_t launch_refine_noalloc(const Geom& g, const GridP& gp, const float2* y, const int64_t* cells, int ncells,
                                 int max_iter, double* theta, int* status, hipStream_t st);

size_t direct_points_ws_bytes(const Geom& g, int npts);
hipError_t launch_direct_points(const Geom& g, const float2* y, const double* theta, int npts, void* ws,
                                double* value, double* grad, double* grad_rx, hipStream_t st);
hipError_t launch_gh_points(const Geom& g, const void* maps, int map_dtype, int interp, const double* theta, int npts,
                            double* value, double* grad, double* grad_rx, hipStream_t st);

}  // namespace gh
