/*
 * gridhop.h - C ABI of the MI355X (gfx950) grid-hopping library.
 *
 * Grid hopping (Monnoyer et al., "Grid Hopping: Accelerating Direct
 * Estimation Algorithms for Multistatic FMCW Radar") evaluates the direct
 * estimator's decision function over a 4D location-velocity grid
 * (x, y, vx, vy) by interpolating each receiver's 2D range-Doppler FFT map
 * instead of computing the scalar products with the model atoms.
 *
 * Conventions shared by every entry point
 *  - Device pointers (prefix d_) are caller-owned HIP device allocations; the
 *    library never allocates device memory (scratch space comes from caller
 *    workspaces whose size the *_workspace_bytes() queries give, or, for
 *    gh_refine_noalloc alone, from a static device array of the library) and retains
 *    no pointer after returning, except a gh_batch object, which keeps its
 *    frame and workspace pointers until gh_batch_destroy.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every call only enqueues work (gh_batch_create alone also synchronises
 *    its stream once); results are valid once the caller has synchronised the
 *    stream, and device faults surface there.
 *  - Arguments are validated on the host before anything is enqueued.  On
 *    error nothing is enqueued, a negative gh_status is returned and
 *    gh_last_error() describes the failure.  No C++ exception crosses the ABI.
 *  - Complex numbers are interleaved (re, im) pairs of float (complex64) or
 *    double.
 *  - Every device array must be 16-byte aligned (hipMalloc and fresh torch
 *    tensors are 256-byte aligned); a misaligned pointer is rejected with
 *    GH_EINVAL.
 *  - Frames: d_y is complex64 [n_rx][n_chirps][n_samples], sample index
 *    fastest: row m of receiver q is chirp m of Y_q in C^{Mc x Ms}
 *    (paper Sec. II, eq. (3)).
 *  - Maps: complex64 [n_rx][N_r][N_d], N_r = pad_range * n_samples range bins,
 *    N_d = pad_doppler * n_chirps Doppler bins, Doppler index fastest.
 *  - Grids: axes (x, y, vx, vy) in metres and metres/second; point i of axis a
 *    is lo[a] + i * (hi[a] - lo[a]) / (n[a] - 1) (n[a] == 1: lo[a]).  The
 *    linear index of (ix, iy, ivx, ivy) is ((ix*Ny + iy)*Nvx + ivx)*Nvy + ivy;
 *    decision volumes are float [Nx][Ny][Nvx][Nvy] in that order.  A "block"
 *    is one location's Nvx*Nvy velocity slab.
 *  - Sensing (paper Sec. II, eqs. (1)-(2), physical FMCW scaling): for
 *    receiver q, R_q = |x - tx| + |x - rx_q|, U_q = <unit(x - tx) +
 *    unit(x - rx_q), v>; cycles per sample f_r = B R_q / (c Ms), cycles per
 *    chirp f_d = f0 Tc U_q / c; map coordinates t_r = f_r N_r, t_d = f_d N_d.
 */
#ifndef GRIDHOP_H
#define GRIDHOP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GH_ABI_VERSION 4
#define GH_MAX_RX 16
#define GH_MAX_SUPPORT 32
#define GH_REFINE_NOALLOC_MAX_CELLS 1024              /* cells per gh_refine_noalloc call */
#define GH_REFINE_NOALLOC_SCRATCH_BYTES (4u << 20)    /* its static device scratch per GPU */

typedef enum {
    GH_OK = 0,
    GH_EINVAL = -1,        /* invalid argument (NULL pointer, bad size, non-finite parameter) */
    GH_EUNSUPPORTED = -2,  /* valid request outside what this library implements */
    GH_EHIP = -3,          /* a HIP runtime call failed (no device, launch failure) */
    GH_EWORKSPACE = -4     /* caller workspace smaller than the matching *_workspace_bytes() */
} gh_status;

/* Interpolation rules.  GH_INTERP_POLAR (the paper's range rule, Sec. IV) is
 * accepted by gh_factored_decision only. */
typedef enum { GH_INTERP_BILINEAR = 0, GH_INTERP_BICUBIC = 1, GH_INTERP_POLAR = 2 } gh_interp;

/* Method of gh_factored_decision. */
typedef enum { GH_FACTOR_DIRECT = 0, GH_FACTOR_GRID_HOPPING = 1 } gh_factor_method;

/* Storage of range-Doppler maps.  GH_MAP_C64: complex64, the map itself.
 * GH_MAP_F16 / GH_MAP_BF16: (re, im) pairs of IEEE binary16 / bfloat16
 * holding Z / (Ms * Mc), an exact power of two that keeps FP16 in range
 * (|Z| <= Ms * Mc * sum |y|); decisions computed from them are rescaled
 * exactly.  The half formats need pad_doppler >= 2. */
typedef enum { GH_MAP_C64 = 0, GH_MAP_F16 = 1, GH_MAP_BF16 = 2 } gh_map_dtype;

typedef enum { GH_GEMM_F32 = 0, GH_GEMM_BF16 = 1 } gh_gemm_dtype;

/* Radar and frame description (paper Sec. II).  Limits: n_samples and
 * n_chirps powers of two in [8, 1024]; pad_range, pad_doppler in {1, 2, 4, 8};
 * N_r and N_d at most 4096; 1 <= n_rx <= GH_MAX_RX; positive finite f0, B,
 * Tc, c.  `centered` selects maps of the centred atoms (index s - (Ms-1)/2,
 * m - (Mc-1)/2), whose interpolation kernel is real; 0 gives plain DFT maps.
 * `rx` is a HOST pointer to n_rx (x, y) pairs in metres, read during the call. */
typedef struct {
    double f0_hz;
    double bandwidth_hz;
    double t_chirp_s;
    double c_mps;
    int32_t n_samples;     /* Ms */
    int32_t n_chirps;      /* Mc */
    int32_t pad_range;     /* P along fast time */
    int32_t pad_doppler;   /* P along slow time */
    int32_t n_rx;          /* K (the paper's Q) */
    int32_t centered;
    double tx[2];
    const double *rx;
} gh_radar;

/* Inclusive 4D grid (paper Sec. III: X_G x V_G).  n[a] >= 1, lo[a] <= hi[a],
 * total points below 2^31. */
typedef struct {
    double lo[4];
    double hi[4];
    int32_t n[4];
} gh_grid;

/* A decision maximum: value and linear grid index (ties -> lowest index). */
typedef struct {
    float value;
    int32_t reserved;
    int64_t index;
} gh_peak;

/* ABI version of the loaded library (GH_ABI_VERSION at build time). */
int gh_abi_version(void);

/* Message of the last failed call on this thread ("" after success).  The
 * pointer stays valid until the next gh_* call on the same thread. */
const char *gh_last_error(void);

/* Range-Doppler maps (paper Sec. III, first step of the indirect method, and
 * Sec. IV, the FFT outputs z that grid hopping interpolates):
 *   Z_q[i][l] = sum_{m<Mc} sum_{s<Ms} Y_q[m][s]
 *               exp(-j 2 pi (i (s - c_s) / N_r + l (m - c_m) / N_d)),
 * c_s = (Ms-1)/2, c_m = (Mc-1)/2 if radar->centered, else 0: the zero-padded
 * (zeros appended, rectangular window) forward 2D DFT.
 * d_y: complex64 [K][Mc][Ms] (read only).  d_maps: [K][N_r][N_d] in the
 * storage `map_dtype` (gh_map_dtype; written; must not overlap d_y).  FP32
 * arithmetic, rounded once to the storage type. */
int gh_rd_maps(const gh_radar *radar, const void *d_y, void *d_maps, int32_t map_dtype, void *stream);

/* Grid-hopping decision (paper Sec. IV, eq. (7)): for every grid point and
 * receiver q, interpolate map q at (t_r, t_d) (bilinear: 2x2 taps; bicubic:
 * 4x4 Keys taps, a = -1/2; periodic in both map axes, with the sign
 * (-1)^(M-1) per period for centred maps) and sum |.|^2 over receivers:
 *   D_gh(x, v) = sum_q |I(Z_q; t_r, t_d)|^2.
 * d_maps: output of gh_rd_maps for the same radar, in storage `map_dtype`.
 * d_decision: float volume (NULL: not written, argmax only).
 * d_block: gh_peak [Nx*Ny], per-location maxima (required).
 * d_argmax: gh_peak [1], global maximum (NULL: not computed).
 * FP32 interpolation and accumulation; geometry in FP64, Doppler coordinate
 * in 32-bit fixed point (exact wrap). */
int gh_decision(const gh_radar *radar, const gh_grid *grid, const void *d_maps, int32_t map_dtype, int32_t interp,
                float *d_decision, gh_peak *d_block, gh_peak *d_argmax, void *stream);

/* Global maximum of per-location peaks (the argmax of eqs. (5)-(6) over the
 * whole grid, from the block maxima gh_decision / gh_direct_decision write):
 * largest value, ties to the lowest index.  d_block: gh_peak [n_block]
 * (1 <= n_block < 2^31); d_argmax: gh_peak [1]. */
int gh_argmax(const gh_peak *d_block, int64_t n_block, gh_peak *d_argmax, void *stream);

/* Workspace of gh_direct_decision in bytes. */
size_t gh_direct_workspace_bytes(const gh_radar *radar, const gh_grid *grid, int32_t gemm_dtype);

/* Direct decision (paper Sec. I and III; the scalar products of eq. (3)'s
 * atoms with the frames, evaluated exactly):
 *   D_dir(x, v) = sum_q | sum_{m,s} Y_q[m][s] exp(-j 2 pi (f_r s + f_d m)) |^2
 * as two contractions per receiver: G_q[x][m] = sum_s Y_q[m][s] conj(a_s(f_r))
 * (range zoom over locations), then per location the Doppler zoom
 * sum_m G_q[x][m] conj(b_m(f_d)) over the velocity slab.  gemm_dtype selects
 * FP32 or BF16 operands (FP32 accumulation either way).
 * d_y: complex64 frames.  d_ws: workspace of gh_direct_workspace_bytes().
 * Outputs as gh_decision. */
int gh_direct_decision(const gh_radar *radar, const gh_grid *grid, const void *d_y, int32_t gemm_dtype,
                       void *d_ws, size_t ws_bytes, float *d_decision, gh_peak *d_block,
                       gh_peak *d_argmax, void *stream);

/* Workspace of gh_bomp_step in bytes. */
size_t gh_bomp_workspace_bytes(const gh_radar *radar, const gh_grid *grid, int32_t use_direct,
                               int32_t gemm_dtype);

/* One Block-OMP iteration (multi-target extension the paper names as future
 * work, Sec. VI):
 *   1. decision on the residual (grid hopping if use_direct == 0, else the
 *      direct decision); the residual is d_resid, or d_y itself when
 *      n_support == 0 (d_resid is then not read).  Grid hopping takes the
 *      maps of the residual: at n_support == 0 gh_rd_maps of d_y, written to
 *      d_maps; later, by linearity of the maps, those of y in d_maps minus
 *      sum_t alpha_t R_t[i] D_t[l], the maps of the fitted atoms in closed
 *      form (Dirichlet sums along range and Doppler in FP64, left in the
 *      workspace by the previous fit; applied in FP32), built in the
 *      workspace (or gh_rd_maps of d_resid there when n_support * N_d
 *      exceeds 4096);
 *   2. select the maximum over the grid excluding the n_support cells already
 *      in d_support; store its index at d_support[n_support];
 *   3. for each receiver, least squares over the n_support + 1 selected cells
 *      with the exact atoms A_q(theta) = b(f_d) (x) a(f_r) of eq. (3):
 *      normal equations in FP64 with the Gram matrix in closed form;
 *      alpha (complex64 [n_support+1][K], row t = cell d_support[t]) to d_alpha;
 *   4. d_resid <- Y - sum_t alpha_t A(theta_t) (FP32).
 * d_y: original frames (read).  d_resid: complex64 [K][Mc][Ms], in/out.
 * d_maps: complex64 map buffer [K][N_r][N_d] (grid hopping: written at
 * n_support == 0 and read by the later iterations of the run, so the caller
 * passes the same buffer, unchanged, throughout; may be NULL when
 * use_direct == 1).  d_ws carries from one iteration to the next the
 * fitted atoms' maps and a counter of the grid maximum that the iteration at
 * n_support == 0 zeroes and the later ones leave at zero: a run starts at
 * n_support == 0 and passes the same workspace throughout.
 * d_support: int64 [max_support], in/out.
 * 0 <= n_support < max_support <= GH_MAX_SUPPORT.  d_selected: gh_peak [1]
 * (NULL: not written), the selected maximum.  Everything stays on the
 * device; no host synchronisation inside.  The same as gh_bomp_select
 * followed by gh_bomp_fit with n_selected = n_support + 1. */
int gh_bomp_step(const gh_radar *radar, const gh_grid *grid, const void *d_y, void *d_resid, void *d_maps,
                 int32_t use_direct, int32_t interp, int32_t gemm_dtype, int64_t *d_support,
                 int32_t n_support, int32_t max_support, void *d_alpha, gh_peak *d_selected,
                 void *d_ws, size_t ws_bytes, void *stream);

/* Steps 1 and 2 of gh_bomp_step alone (arguments as there): after it,
 * d_support[0 .. n_support] holds the selection.  Lets a caller start work
 * that needs only the selected cells (gh_refine) before the fit. */
int gh_bomp_select(const gh_radar *radar, const gh_grid *grid, const void *d_y, const void *d_resid,
                   void *d_maps, int32_t use_direct, int32_t interp, int32_t gemm_dtype, int64_t *d_support,
                   int32_t n_support, int32_t max_support, gh_peak *d_selected, void *d_ws, size_t ws_bytes,
                   void *stream);

/* Steps 1 and 2 of gh_bomp_step at n_support == 0 (grid hopping) taken from a
 * grid-hopping decision the caller has already made on the frame itself, so
 * that a caller who needs both that decision (its volume, say) and Block-OMP
 * computes the frame's maps and the first sweep once.  Preconditions (the
 * caller's): the run's d_maps holds gh_rd_maps of d_y (complex64), the buffer
 * later passed to gh_bomp_select / gh_bomp_step, and d_block holds the
 * per-location maxima (gh_peak [Nx*Ny]) of gh_decision over the same grid with
 * the same interp, computed from those maps.  Takes their maximum (the
 * argmax of eqs. (5)-(6), ties to the lowest index, as gh_argmax), writes
 * its index to d_support[0] and, when d_selected is non-NULL, the maximum
 * itself to *d_selected, and readies d_ws (of gh_bomp_workspace_bytes(radar,
 * grid, 0, any gemm_dtype) bytes) for the later selections; one launch.  The
 * run then continues with gh_bomp_fit(n_selected = 1).  max_support and
 * interp as in gh_bomp_step. */
int gh_bomp_seed(const gh_radar *radar, const gh_grid *grid, int32_t interp, const gh_peak *d_block,
                 int64_t *d_support, int32_t max_support, gh_peak *d_selected, void *d_ws, size_t ws_bytes,
                 void *stream);

/* Steps 3 and 4 of gh_bomp_step alone: least squares over the n_selected
 * cells d_support[0 .. n_selected) (1 <= n_selected <= max_support <=
 * GH_MAX_SUPPORT), alpha (complex64 [n_selected][K]) to d_alpha, and
 * d_resid <- Y - sum_t alpha_t A(theta_t); the fitted atoms' maps are left
 * in the workspace for the next selection.  d_ws: the run's workspace, of
 * gh_bomp_workspace_bytes(radar, grid, use_direct, gemm_dtype) bytes for any
 * use_direct and gemm_dtype (this call uses the part they share); it must not
 * be in use by a gh_bomp_select or gh_bomp_step still running on another
 * stream. */
int gh_bomp_fit(const gh_radar *radar, const gh_grid *grid, const void *d_y, void *d_resid, const int64_t *d_support,
                int32_t n_selected, int32_t max_support, void *d_alpha, void *d_ws, size_t ws_bytes, void *stream);

/* Workspace of gh_refine in bytes for n_cells (1..65535) starting cells; 0 on
 * invalid arguments (see gh_last_error). */
size_t gh_refine_workspace_bytes(const gh_radar *radar, const gh_grid *grid, int32_t n_cells);

/* Off-grid refinement of the direct decision (not in the paper): starting at
 * each cell (int64 linear grid index, device), the converged local maximum of
 * D_dir over continuous (x, y, vx, vy) within one grid step per axis (the box
 * around the cell), by projected Newton ascent with analytic gradient and
 * Hessian: a coordinate next to a face of the box whose gradient points
 * outwards is put on that face, the others take the Newton step of the
 * problem restricted to them (eigenvalues replaced by -|lambda|); the step is
 * halved until the decision does not decrease (at most 16 candidates).  Stops
 * when the projected step, or the accepted move, is below 1e-7 grid steps in
 * every coordinate (KKT on the box), or after max_iter (1..100) iterations.
 * An axis with one grid point is held.  d_ws: workspace of
 * gh_refine_workspace_bytes() (barrier counters
 * and partial moments; its contents need no initialisation; may be NULL when
 * n_cells == 0, which enqueues nothing and leaves d_status unwritten).
 * d_theta: double [n_cells][4] out; NaN marks a cell whose cooperating
 * workgroups failed to meet within a bounded wait (at least 0.2 s; possible
 * only when other work holds the device's compute units for that long).
 * d_status: int32 [1] out (NULL: not written), the number of such NaN cells
 * (0 when every estimate is valid); read it after synchronising the stream.
 * FP64 throughout: phases in 64-bit fixed point (exact modulo one cycle),
 * phase factors, moments and the Newton solve in FP64. */
int gh_refine(const gh_radar *radar, const gh_grid *grid, const void *d_y, const int64_t *d_cells,
              int32_t n_cells, int32_t max_iter, void *d_ws, size_t ws_bytes, double *d_theta,
              int32_t *d_status, void *stream);

/* gh_refine for callers that cannot allocate device memory or own a workspace
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same refinement and results, with the scratch (barrier
 * counters and partial moments) taken from a static device array of
 * GH_REFINE_NOALLOC_SCRATCH_BYTES inside the library instead of d_ws.  Every
 * GPU the library runs this on holds one such array until the process ends.
 * Allocates nothing and calls no allocating routine; it clears what must
 * start at zero with a kernel, so it can be captured.  Cells that need more
 * partial-moment slots at once than the array holds are refined by several
 * launches.  n_cells: 0..GH_REFINE_NOALLOC_MAX_CELLS (more: GH_EUNSUPPORTED,
 * nothing enqueued); other arguments as gh_refine.  Every call on one GPU
 * shares that GPU's array: calls that may overlap in time on one GPU (other
 * streams, other threads, other processes' contexts excepted) race and give
 * undefined results; serialise them (one stream, or events). */
int gh_refine_noalloc(const gh_radar *radar, const gh_grid *grid, const void *d_y, const int64_t *d_cells,
                      int32_t n_cells, int32_t max_iter, double *d_theta, int32_t *d_status, void *stream);

/* Decisions at continuous points, with gradients (differentiation axis; not
 * in the paper).  For each point theta = (x, y, vx, vy) (d_theta: double
 * [n_points][4], device):
 *   d_value[i]             D(theta_i)                       (double [n_points])
 *   d_grad[i][a]           dD/dtheta_a                      (double [n_points][4]; NULL: not computed)
 *   d_grad_rx[i][q][b]     dD/d(rx_q)_b, receiver positions (double [n_points][K][2]; NULL: not computed)
 * from dD/dp = sum_q 2 Re(conj(c_q) dc_q/dp) through the sensing functions of
 * eqs. (1)-(2).  1 <= n_points <= 65535 (0: nothing is enqueued).  A
 * non-finite theta gives non-finite outputs. */

/* Workspace of gh_direct_points in bytes (0 on invalid arguments). */
size_t gh_direct_points_workspace_bytes(const gh_radar *radar, int32_t n_points);

/* Direct decision at points (Sec. I and III, scalar products with the atoms of
 * eq. (3)): c_q = sum_{m,s} Y_q[m][s] exp(-j 2 pi (f_r s + f_d m)) with the
 * moments M_10, M_01 (sample- and chirp-weighted sums) for the gradient.
 * d_y: complex64 frames.  FP32 per chirp, FP64 beyond. */
int gh_direct_points(const gh_radar *radar, const void *d_y, const double *d_theta, int32_t n_points,
                     double *d_value, double *d_grad, double *d_grad_rx, void *d_ws, size_t ws_bytes,
                     void *stream);

/* Grid-hopping decision at points (Sec. IV, eq. (7)): the interpolated map
 * values I_q at (t_r, t_d) in FP64 coordinates (bilinear or Keys bicubic,
 * periodic with the centring sign), with dI/dt from the kernel derivative
 * (bilinear: piecewise constant, one-sided at map nodes).  d_maps: output of
 * gh_rd_maps in storage map_dtype. */
int gh_gh_points(const gh_radar *radar, const void *d_maps, int32_t map_dtype, int32_t interp,
                 const double *d_theta, int32_t n_points, double *d_value, double *d_grad, double *d_grad_rx,
                 void *stream);

/* ---- Factorised decisions (paper Sec. III, eqs. (5)-(6), and Sec. IV) ------
 * The paper's own sequence: the location first, from the energy of the
 * per-chirp range correlations,
 *   E(x) = sum_q sum_m |<Y_q[m], a(f_r,q(x))>|^2,           x^ = argmax over the location grid,
 * then the velocity at x^ from each receiver's chirp sequence of range
 * correlations there, g_q[m],
 *   V(v) = sum_q |<g_q, b(f_d,q(x^, v))>|^2,                 v^ = argmax over the velocity grid
 * (the atom of eq. (6) read as the Doppler atom b).  Grid hopping replaces the
 * scalar products of (5) by a range interpolation of per-chirp range spectra
 * (gh_range_spectra) and those of (6) by the nearest bin, round(t_d), of the
 * zero-padded FFT over chirps of the interpolated g_q (Sec. IV: a single
 * index in Doppler). */

/* Per-chirp zero-padded range spectra (the range FFT of Sec. IV, before any
 * transform over chirps): spectra[q][i][m] = sum_s Y_q[m][s]
 * exp(-j 2 pi i (s - c_s) / N_r), c_s as in gh_rd_maps.  d_y: complex64
 * [K][Mc][Ms]; d_spectra: complex64 [K][N_r][Mc] (written; must not overlap
 * d_y).  FP32. */
int gh_range_spectra(const gh_radar *radar, const void *d_y, void *d_spectra, void *stream);

/* Workspace of gh_factored_decision in bytes (0 on invalid arguments). */
size_t gh_factored_workspace_bytes(const gh_radar *radar, const gh_grid *grid, int32_t method);

/* Factorised decision, eqs. (5)-(6).
 * method GH_FACTOR_DIRECT: d_input = the frames (complex64 [K][Mc][Ms]); the
 *   correlations of (5) by the range zoom of gh_direct_decision (gemm_dtype
 *   F32 or BF16 operands), those of (6) exactly (FP32 per chirp, fixed-point
 *   phases); range_interp ignored.
 * method GH_FACTOR_GRID_HOPPING: d_input = gh_range_spectra of the frames;
 *   range_interp = GH_INTERP_BILINEAR, GH_INTERP_BICUBIC (Keys, a = -1/2) or
 *   GH_INTERP_POLAR: the three bins around the nearest one, weighted by the
 *   circle through their three atoms (angle theta per bin from the atoms'
 *   chord lengths, |f(1) - f(-1)|^2 / |f(1) - f(0)|^2 = 2 (1 + cos theta));
 *   taps wrap with the centring sign; gemm_dtype ignored.
 * d_loc: float [Nx][Ny], E(x) (NULL: not written).  d_vel: float [Nvx][Nvy],
 * V(v) at the selected location (NULL: not written).  d_result: gh_peak [2]:
 * [0] = (E(x^), location index ix*Ny + iy), [1] = (V(v^), linear 4D grid
 * index of (x^, v^)); ties to the lowest index.  Everything stays on the
 * device. */
int gh_factored_decision(const gh_radar *radar, const gh_grid *grid, int32_t method, int32_t range_interp,
                         int32_t gemm_dtype, const void *d_input, void *d_ws, size_t ws_bytes, float *d_loc,
                         float *d_vel, gh_peak *d_result, void *stream);

/* ---- Batches of frames (batching axis; not in the paper) -------------------
 * Many frames of different shapes (radar, grid) decided together: their maps
 * (gh_rd_maps), grid-hopping decisions (gh_decision) and per-frame argmax,
 * each step as one persistent launch over all frames that reads a
 * frame-descriptor table in device memory.  A gh_batch is a host object made
 * once per batch layout; unlike every other entry point it RETAINS the frame
 * and workspace pointers it was created with (until gh_batch_destroy), so a
 * run only launches kernels and can be captured in a HIP graph and replayed:
 * it enqueues no memset or copy and needs nothing reset between runs. */

/* One frame of a batch.  radar->rx is read during gh_batch_create. */
typedef struct {
    gh_radar radar;
    gh_grid grid;
    const void *d_y;      /* complex64 [K][Mc][Ms] (read at every run) */
    float *d_decision;    /* float volume of the frame's grid, or NULL (not written) */
    gh_peak *d_block;     /* gh_peak [Nx*Ny] per-location maxima (required) */
} gh_frame;

typedef struct gh_batch gh_batch;   /* opaque */

/* Launch shape of a batch (gh_batch_get_info). */
typedef struct {
    int32_t n_frames;
    int32_t interp;
    int32_t units[3];           /* work units of the range, Doppler and sweep launches */
    int32_t workgroups[3];      /* persistent grid sizes in use (gh_batch_tune) */
    int32_t max_workgroups[3];  /* workgroups resident at once (occupancy x compute units) */
    int32_t sweep_waves;        /* waves per sweep workgroup: 1, 2 or 4 */
    int32_t column_height;      /* compiled vx points per lane of the sweep */
    int32_t sweep_locations;    /* consecutive locations per sweep work unit (gh_batch_tune_tiles) */
    int32_t range_chirps;       /* chirps per range workgroup requested (0: each frame's planner) */
    int32_t doppler_rows;       /* range rows per Doppler workgroup requested (0: each frame's planner) */
    int64_t points;             /* grid points over all frames */
    int64_t workspace_bytes;    /* bytes of the workspace the batch uses */
} gh_batch_info;

/* Workspace of a batch in bytes: the descriptor table and every frame's
 * complex64 maps.  0 on invalid frames (see gh_last_error). */
size_t gh_batch_workspace_bytes(const gh_frame *frames, int32_t n_frames);

/* Validate 1 <= n_frames <= 65535 frames (host array), lay out d_ws and upload
 * the descriptor table on `stream`, then synchronise that stream once (this
 * call blocks; gh_batch_run never does).  Per frame: the limits of gh_rd_maps
 * and gh_decision, N_d >= 16, Nvy <= 64 and ceil(Nvx / floor(64 / Nvy)) <= 32
 * (a lane's share of the velocity slab); one wave's LDS slice, 768 bytes of
 * per-receiver coordinate records plus the Doppler table of the largest N_d
 * (16 bytes per bin bilinear, 32 bicubic), must fit in 64 KB, and so must the
 * map passes' buffers (GH_EUNSUPPORTED otherwise: N_d = 4096 bilinear,
 * N_d >= 2048 bicubic).  interp: GH_INTERP_* for every frame.  d_ws must hold
 * gh_batch_workspace_bytes(); its contents belong to the batch until
 * gh_batch_destroy.  *batch receives the new object (NULL on error). */
int gh_batch_create(const gh_frame *frames, int32_t n_frames, int32_t interp, void *d_ws, size_t ws_bytes,
                    gh_batch **batch, void *stream);

/* Persistent grid sizes (the batch's tuning knobs): workgroups of the range,
 * Doppler and sweep launches (0 keeps the current value; defaults: as many
 * as are resident at once), and waves per sweep workgroup (1, 2 or 4; 0
 * keeps).  Any positive count is correct; launches clamp to their units. */
int gh_batch_tune(gh_batch *batch, int32_t range_workgroups, int32_t doppler_workgroups, int32_t sweep_workgroups,
                  int32_t sweep_waves);

/* Tiles of the batch's launches (the autotuner's other knobs): chirps per
 * range-pass workgroup and range rows per Doppler-pass workgroup (0: each
 * frame's planner; else a power of two up to 4096, clamped per frame to what
 * a workgroup holds), and consecutive locations per sweep work unit (1..64;
 * 0 keeps).  Re-plans every frame's work units, uploads the descriptor table
 * on `stream` and synchronises it (not for use inside a graph capture); the
 * range and Doppler workgroup counts go back to their resident maximum.
 * Results do not depend on the tiles.  GH_EUNSUPPORTED if a map pass would
 * need more than 64 KB of LDS. */
int gh_batch_tune_tiles(gh_batch *batch, int32_t range_chirps, int32_t doppler_rows, int32_t sweep_locations,
                        void *stream);

int gh_batch_get_info(const gh_batch *batch, gh_batch_info *info);

/* One pass over every frame: maps, decision (volume when d_decision was given,
 * block maxima always) and d_argmax[f] = the frame's maximum (gh_peak
 * [n_frames], ties to the lowest index; NULL: not computed).  Results equal
 * gh_rd_maps + gh_decision + gh_argmax per frame.  Runs on the device the
 * batch was created on. */
int gh_batch_run(const gh_batch *batch, gh_peak *d_argmax, void *stream);

/* Device address of frame f's complex64 maps [K][N_r][N_d] inside the batch
 * workspace (valid after a run, until the next run overwrites them; for
 * gh_gh_points or gh_decision on one frame). */
int gh_batch_frame_maps(const gh_batch *batch, int32_t frame, void **d_maps);

/* Free the host object (NULL is a no-op).  Work already enqueued is unaffected. */
void gh_batch_destroy(gh_batch *batch);

#ifdef __cplusplus
}
#endif

#endif /* GRIDHOP_H */
