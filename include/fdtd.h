/*
 * fdtd.h -- C ABI of the MI355X (gfx950) time-reversible FDTD gradient library.
 *
 * Method: Mahlau, Berg, Rosenhahn, "Numerical field optimization for enhanced
 * efficiency in time-reversible gradient computation of open-source
 * GPU-accelerated FDTD simulations" (arXiv 2603.24027).
 *
 *   - forward: 3-D Yee leapfrog with convolutional-PML absorbing faces, time
 *     step from the Courant number by Eq. 1; the tangential fields on the
 *     interface slices between the interior and the PML are recorded
 *     (Section 2, first paragraph);
 *   - recording is compressed by a smaller storage type (Section 2, bit-width
 *     reduction) and by keeping every k-th step with linear interpolation in
 *     between (Section 2, the paragraph after Eq. 1; Fig. 1b);
 *   - backward: the simulation runs backwards in time from its final state
 *     through the lossless interior, the recorded interface fields are
 *     injected back as sources (Section 1, Section 2), and the exact
 *     discrete adjoint accumulates dL/deps per design cell in FP64.
 *
 * Units are normalised: cell size 1, c = 1, eps0 = mu0 = 1, mu = 1.
 * Grid arrays are float32, structure-of-arrays, x fastest:
 *     idx(i, j, k) = i + nx * (j + ny * k).
 * Boxes are half-open index ranges [lo, hi) given as (x, y, z).
 *
 * Ownership: every pointer is owned by the caller.  The library never
 * allocates, frees or synchronises device memory; it only launches kernels
 * on the caller's HIP stream.  Host pointers (source signal and profiles)
 * are read before the call returns.
 *
 * Errors: every entry point returns 0 on success or a negative FDTD_E* code;
 * fdtd_last_error() gives a message for the calling thread.  All argument
 * validation happens before the first HIP call, so invalid arguments are
 * reported the same way with or without a GPU.  No C++ exception crosses
 * this interface.
 */
#ifndef FDTD_MI355X_H
#define FDTD_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define FDTD_API __attribute__((visibility("default")))
#else
#define FDTD_API
#endif

#define FDTD_OK          0
#define FDTD_EINVAL     -1   /* malformed argument (null pointer, size, enum)            */
#define FDTD_ECFL       -2   /* Courant number outside (0, 1] (Eq. 1 stability)          */
#define FDTD_EREGION    -3   /* source / detector / design box not inside the interior   */
#define FDTD_ESTORE     -4   /* storage config invalid, or record from another problem   */
#define FDTD_ESTATE     -5   /* backward on a consumed record (fields already reversed)  */
#define FDTD_EHIP       -6   /* a HIP runtime call failed                                */
#define FDTD_ENONFINITE -7   /* non-finite loss (reported by bindings that read it)      */

/* Storage types of the recorded interface fields (Section 2). */
#define FDTD_STORE_FP32              0   /* plain copy                                     */
#define FDTD_STORE_FP16              1   /* IEEE binary16, round to nearest even           */
#define FDTD_STORE_BF16              2   /* bfloat16, round to nearest even                */
#define FDTD_STORE_FP8_E4M3_SCALED   3   /* OCP E4M3 (max 448, no inf) of x / s with one
                                            power-of-two s per (kept step, face, component):
                                            s = 2^e, e the smallest integer such that
                                            448 * 2^e >= max|x|, clamped to [-126, 127]     */
/* The unscaled 8-bit types compared in Section 3 (Fig. 3): eXmY = exponent and
 * mantissa bits; "fn" = finite with NaN; "fnuz" = finite, NaN, unsigned zero;
 * b11 = exponent bias 11.  Values past the largest finite one become inf (IEEE
 * style) or NaN, as a plain (non-saturating) conversion gives. */
#define FDTD_STORE_FP8_E4M3B11FNUZ   4   /* bias 11, max 30, smallest subnormal 2^-13      */
#define FDTD_STORE_FP8_E5M2FNUZ      5   /* bias 16, max 57344                              */
#define FDTD_STORE_FP8_E4M3FNUZ      6   /* bias 8, max 240                                 */
#define FDTD_STORE_FP8_E4M3          7   /* IEEE style, bias 7, max 240                     */
#define FDTD_STORE_FP8_E3M4          8   /* IEEE style, bias 3, max 15.5                    */
#define FDTD_STORE_FP8_E4M3FN        9   /* OCP E4M3 without a scale, max 448               */

#define FDTD_MAX_PML 64

/*
 * Problem statement: grid with PML faces, permittivity map, source, detector
 * and Courant number (Section 2 and Eq. 1; PML from Section 1).
 *
 *   nx, ny, nz      full grid in cells, PML included (each >= 1; 24 * S < 2^31 for the
 *                   component stride S of fdtd_store_info_t.fields_bytes,
 *                   and the two copies of the PML auxiliaries below 2 GiB)
 *   pml             PML thickness P on all six faces (0 <= P <= FDTD_MAX_PML,
 *                   2P < each extent); the interior I is [P, n-P) on each axis
 *   steps           T >= 1 time steps
 *   boundary        0: fields are zero outside the array; 1: periodic (needs P = 0)
 *   courant         C in (0, 1]; dt = C / sqrt(3)  (Eq. 1)
 *   pml_order       polynomial grading m >= 1
 *   pml_sigma_scale sigma_max = scale * 0.8 (m + 1)
 *   pml_kappa_max   >= 1
 *   pml_alpha_max   >= 0 (complex-frequency shift, linear from the interface)
 *   src_comp        0, 1, 2 = Jx, Jy, Jz
 *   src_lo, src_hi  source box (inside I)
 *   src_wave        host, T floats: J^n sampled at t = (n + 1/2) dt
 *   src_profile     host, box-volume floats in [z][y][x] order: J on the box
 *                   at step n is src_wave[n] * src_profile[...]
 *   det_lo, det_hi  detector box D (inside I)
 *   des_lo, des_hi  design box (inside I): dL/deps is returned for these cells
 *   loss            0: L = sum_{n<T} sum_{p in D} |E^{n+1}(p)|^2;
 *                   1, 2, 3: L = sum_{n<T} sum_{p in D} (E^{n+1}(p) x H^{n+1/2}(p))_{x, y, z},
 *                   the Poynting flux along x, y or z (Section 3's transmission
 *                   metric), E and H taken at the same cell index
 *   msrc_comp       0, 1, 2 = Mx, My, Mz: an optional magnetic current, dH/dt = -curl E - M
 *                   (with J, the two sheets of a total-field/scattered-field plane wave)
 *   msrc_lo, msrc_hi  its box (inside I); an empty box means none
 *   msrc_wave       host, T floats: M^n (enters the H update of step n); NULL if none
 *   msrc_profile    host, box-volume floats in [z][y][x] order; NULL if none
 */
typedef struct {
    int32_t nx, ny, nz;
    int32_t pml;
    int32_t steps;
    int32_t boundary;
    double  courant;
    int32_t pml_order;
    double  pml_sigma_scale;
    double  pml_kappa_max;
    double  pml_alpha_max;
    int32_t src_comp;
    int32_t src_lo[3], src_hi[3];
    const float* src_wave;
    const float* src_profile;
    int32_t det_lo[3], det_hi[3];
    int32_t des_lo[3], des_hi[3];
    int32_t loss;
    int32_t msrc_comp;
    int32_t msrc_lo[3], msrc_hi[3];
    const float* msrc_wave;
    const float* msrc_profile;
} fdtd_problem_t;

/* Recorder configuration: storage type (FDTD_STORE_*) and subsampling k >= 1.
 * Kept steps: K = {T-1, T-1-k, ...} (ceil(T/k) of them); the reverse pass
 * rebuilds the others by interpolation in time between kept steps, with an
 * exact zero at step -1:
 *   interp 0 or 1: linear between the two kept neighbours (Section 2; Fig. 1b);
 *   interp 3:      cubic, the Lagrange polynomial through the four nearest nodes
 *                  (kept steps and the zero anchor; n in the middle interval,
 *                  shifted inward at the ends of the run; linear when fewer than
 *                  four nodes exist).  An option beyond the paper's method: it only
 *                  changes how fdtd_backward rebuilds the shell, not what is stored.
 */
typedef struct {
    int32_t dtype;
    int32_t k;
    int32_t interp;
} fdtd_store_cfg_t;

#define FDTD_INTERP_LINEAR 1
#define FDTD_INTERP_CUBIC  3

/* Sizes the caller must allocate (bytes) and storage accounting. */
typedef struct {
    uint64_t cells;             /* nx * ny * nz                                          */
    uint64_t slices;            /* ceil(T / k) kept steps                                */
    uint64_t values_per_slice;  /* 4 * (my*mz + mx*mz + mx*my); 0 when P = 0             */
    uint64_t payload_bytes;     /* slices * values_per_slice * storage bytes (Fig. 3)    */
    uint64_t scale_bytes;       /* 12 float scales per kept step (FP8 only)              */
    uint64_t store_bytes;       /* size of the store buffer (payload, padding, scales)   */
    uint64_t fields_bytes;      /* 6 * S * 4: Ex Ey Ez Hx Hy Hz, component c of cell i at
                                   float c * S + i; S = fields_bytes / 24 >= cells         */
    uint64_t psi_bytes;         /* forward PML auxiliaries (H side in two copies)        */
    uint64_t adj_psi_bytes;     /* backward PML auxiliaries (two copies, ping-pong)      */
    uint64_t workspace_bytes;   /* coefficient tables, source profile, loss partials,
                                   recorder staging, the tiles' launch order, and two
                                   more field buffers (the ping-pong partners of fields
                                   and adj_fields), in that order                        */
    uint64_t design_cells;      /* cells of the design box (length of the gradient)      */
} fdtd_store_info_t;

/* Layout of the store buffer (read it only for inspection; the backward call
 * decodes it itself).  Kept step j (j = 0 .. slices-1 holds time step T-1-j*k)
 * starts at byte j * S, S = values_per_slice * storage bytes rounded up to a
 * multiple of 256.  Within a kept step, 12 (face, component) blocks follow each
 * other, each over the interior extent of the face's two other axes:
 *    0, 1  x-low face,  index P-1:    Hy, Hz   as [z][y]   (my * mz values each)
 *    2, 3  y-low face,  index P-1:    Hz, Hx   as [z][x]   (mx * mz)
 *    4, 5  z-low face,  index P-1:    Hx, Hy   as [y][x]   (mx * my)
 *    6, 7  x-high face, index nx-P:   Ey, Ez   as [z][y]
 *    8, 9  y-high face, index ny-P:   Ez, Ex   as [z][x]
 *   10, 11 z-high face, index nz-P:   Ex, Ey   as [y][x]
 * (H^{n+1/2} on the low faces and E^n on the high faces of time step n.)  For
 * FDTD_STORE_FP8_E4M3_SCALED the float scales follow at byte slices * S, 12
 * per kept step in block order. */

/* Host-side token tying a backward call to the forward call that recorded the store. */
typedef struct {
    uint64_t problem_hash;
    int32_t  dtype;
    int32_t  k;
    int32_t  steps;
    int32_t  consumed;
} fdtd_record_t;

/* Sizes and storage accounting for a problem and recorder configuration.
 * Host only; no HIP call.  Returns FDTD_E* on an invalid problem or config. */
FDTD_API int store_config(const fdtd_problem_t* prob, const fdtd_store_cfg_t* cfg, fdtd_store_info_t* info);

/*
 * Forward simulation with interface recording (Section 2).
 *   eps         device, cells floats: relative permittivity per cell (> 0), used
 *               by Ex, Ey, Ez of that cell index
 *   fields      device, fields_bytes: out, E^T then H^{T-1/2} (zeroed by the call first)
 *   psi         device, psi_bytes: PML auxiliaries (scratch, zeroed by the call)
 *   store       device, store_bytes: out, recorded interface fields
 *   workspace   device, workspace_bytes: scratch (the call writes the CPML
 *               coefficient table and source profiles into it itself; nothing in it
 *               is needed after the call's kernels end)
 *   loss        device, 1 double: out, L
 *   loss_series device, T doubles or NULL: out, per-step terms of L
 *   rec         host: out, token for fdtd_backward
 *   stream      hipStream_t (NULL = default stream)
 * Asynchronous: returns after enqueueing; nothing is synchronised.  The host
 * arrays of the problem (source signal and profiles) are read before the call
 * returns: the few values they contribute travel as kernel arguments, so no
 * host memory is read by the device afterwards.
 * Tile shapes, and whether the forward advances one or two time steps per sweep,
 * are chosen from the grid; the environment variables FDTD_TILE_Y/Z (forward),
 * FDTD_ADJ_TILE_Y/Z and FDTD_REV_TILE_Y/Z (the two reverse sweeps) override the
 * shapes for tuning (Y: 4 or 8 rows; Z: planes per tile, 4 or 8, and 5 or 6 for
 * the reversal with 4 rows), FDTD_FWD_STEPS (1 or 2) the steps per forward sweep
 * and FDTD_FWD2_TILE_Z (8 or 16) the depth of the two-step tiles, FDTD_TILE_ORDER
 * (1: the default order of small grids, 2: octants) the launch order of every
 * sweep; results do not depend on them beyond FP32 rounding order (on the launch
 * order not at all).
 */
FDTD_API int fdtd_forward(const fdtd_problem_t* prob, const fdtd_store_cfg_t* cfg,
                 const float* eps, float* fields, float* psi, void* store, void* workspace,
                 double* loss, double* loss_series, fdtd_record_t* rec, void* stream);

/*
 * fdtd_forward for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops or harnesses that forbid hipMalloc): the same
 * arguments, kernels and results as fdtd_forward (bit for bit), without the
 * workspace argument.  Its workspace is a device array of the library,
 * FDTD_NOALLOC_SCRATCH_BYTES long, which every GPU the library runs on holds
 * from the library's load until the process ends; the call allocates nothing
 * (no hipMalloc, no graph instantiation: it always enqueues its launches
 * directly).
 *   Limit: workspace_bytes - fields_bytes of fdtd_store_info_t (the tables, loss
 *   partials, recorder staging and one ping-pong field buffer) must not exceed
 *   FDTD_NOALLOC_SCRATCH_BYTES (a 128^3 grid fits); larger problems return
 *   FDTD_EINVAL before any HIP call.
 *   Sharing: every call on one GPU uses that GPU's one array, and nothing in it
 *   outlives the call's kernels: calls whose kernels overlap on one GPU (other
 *   streams, other host threads) race and must be serialised by the caller.
 * The record it returns feeds fdtd_backward as fdtd_forward's does.
 */
#define FDTD_NOALLOC_SCRATCH_BYTES (64u << 20)
FDTD_API int fdtd_forward_noalloc(const fdtd_problem_t* prob, const fdtd_store_cfg_t* cfg,
                 const float* eps, float* fields, float* psi, void* store,
                 double* loss, double* loss_series, fdtd_record_t* rec, void* stream);

/*
 * Time-reversed gradient pass (Section 1: backwards from the final step with
 * one extra simulation; Section 2: interface fields injected as sources).
 *   fields      device, in: the final state left by fdtd_forward; destroyed
 *   store       device, in: the record written by fdtd_forward
 *   workspace   device, workspace_bytes: scratch (need not be the forward's buffer)
 *   adj_fields  device, fields_bytes: scratch for the adjoint fields
 *   adj_psi     device, adj_psi_bytes: scratch for the adjoint PML auxiliaries
 *   grad_scale  device, 1 double or NULL: the gradient is multiplied by it
 *               (the upstream derivative in a chained rule); NULL means 1
 *   grad_eps    device, design_cells doubles: out, dL/deps on the design box in
 *               [z][y][x] order, accumulated over time in FP64
 *   rec         host, in/out: must come from the matching fdtd_forward; marked
 *               consumed (a second backward on it returns FDTD_ESTATE)
 * Asynchronous like fdtd_forward.  Whether the reverse primal pass takes one or
 * two time steps per sweep is chosen from the grid; FDTD_REV_STEPS (1 or 2)
 * overrides it and FDTD_REV2_TILE_Z (8 or 16) sets the depth of the two-step
 * tiles.  The two forms give the same gradient up to FP32 rounding order.
 */
FDTD_API int fdtd_backward(const fdtd_problem_t* prob, const fdtd_store_cfg_t* cfg,
                  const float* eps, float* fields, const void* store, void* workspace,
                  float* adj_fields, float* adj_psi, const double* grad_scale,
                  double* grad_eps, fdtd_record_t* rec, void* stream);

/*
 * The recorder's codec on its own (Section 2, bit-width reduction): encodes
 * n_blocks blocks of block_len float32 values (device, contiguous) the way
 * the forward pass stores one (kept step, face, component) block, writes the
 * codes (device, n_blocks * block_len * storage bytes) and, for FP8, one
 * float scale per block (device, may be NULL otherwise), then decodes them
 * back into `decoded` (device, float32).
 */
FDTD_API int fdtd_codec_roundtrip(int32_t dtype, const float* values, int64_t n_blocks, int64_t block_len,
                         void* codes, float* scales, float* decoded, void* stream);

/*
 * Per-kernel timing with HIP events recorded around every launch on the
 * caller's stream.  fdtd_timing_enable(1) clears the counters and starts
 * recording; fdtd_timing_read synchronises on the recorded events and fills
 * up to max_kinds entries, returning the number filled (or a negative code).
 */
typedef struct {
    char     name[32];
    uint64_t launches;
    double   total_ms;
} fdtd_kernel_time_t;

FDTD_API int fdtd_timing_enable(int32_t enable);

/*
 * Launch-sequence replay.  By default a forward or backward call whose
 * problem, store configuration, buffer pointers and device equal those of an
 * earlier call replays that call's kernel sequence as one HIP graph (captured
 * once, up to 16 kept) instead of enqueuing T launches from the host; the
 * kernels and their results are the same.  A 17th distinct call evicts the
 * oldest graph, and that call first waits (on the host) for the evicted graph's
 * last launch to finish.  fdtd_set_graphs(0) enqueues every launch directly.
 * Per-kernel timing always enqueues directly.
 */
FDTD_API int fdtd_set_graphs(int32_t enable);
FDTD_API int fdtd_timing_read(fdtd_kernel_time_t* out, int32_t max_kinds);

FDTD_API const char* fdtd_strerror(int code);
FDTD_API const char* fdtd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FDTD_MI355X_H */
