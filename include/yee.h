/*
 * yee.h -- C ABI of the MI355X (gfx950) Yee FDTD time-step library.
 *
 * The library advances a 3-D staggered-grid (Yee) electromagnetic field in
 * time: per step one H half-update (forward differences of E) and one E
 * half-update (backward differences of H) with per-cell lossy material
 * coefficients, convolutional PML (CPML) layers, PEC faces and PEC masks,
 * soft point sources, and probes with an FP64 running DFT.
 *
 * Source of the definitions.  The paper this library accompanies (radar
 * ray-meta-data simulation; Sections II.A-II.E, Eqs. 1-7) contains no
 * full-wave solver: no grid, field update or time-stepping scheme.  The
 * operation is therefore the textbook one, and each entry point below names
 * it:  Yee, IEEE Trans. Antennas Propag. 14(3), 1966 (staggering, leapfrog);
 * Taflove & Hagness, "Computational Electrodynamics: The FDTD Method",
 * ch. 3 (lossy Ca/Cb form) and ch. 7 (CPML); Roden & Gedney, Microwave Opt.
 * Technol. Lett. 27(5), 2000 (CPML recursion).
 *
 * Conventions shared by every call
 *  - Return value: YEE_OK (0) or a negative yee_status.  No call aborts or
 *    throws; yee_last_error() returns a thread-local message for the last
 *    failing call on this thread.
 *  - Device memory: the caller owns it.  yee_footprint() says how many bytes
 *    one context needs; the caller allocates one device buffer of at least
 *    that size (256-byte aligned) and hands it to yee_bind_workspace().  The
 *    library never allocates device memory and never frees the caller's.
 *  - Host arrays passed in are copied before the call returns.
 *  - Streams: `stream` is a hipStream_t passed as void* (NULL = the null
 *    stream).  Calls that launch work are asynchronous on that stream unless
 *    documented as synchronizing.
 *  - Grid indices: cell (i, j, k), 0 <= i < nx, 0 <= j < ny, 0 <= k < nz.
 *    Components sit at the Yee positions
 *        Ex ((i+1/2)dx, j dy, k dz)    Hx (i dx, (j+1/2)dy, (k+1/2)dz)
 *        Ey (i dx, (j+1/2)dy, k dz)    Hy ((i+1/2)dx, j dy, (k+1/2)dz)
 *        Ez (i dx, j dy, (k+1/2)dz)    Hz ((i+1/2)dx, (j+1/2)dy, k dz)
 *    Host field arrays are [nz][ny][nx] doubles (x fastest) covering the
 *    samples with 0 <= i < nx, 0 <= j < ny, 0 <= k < nz.  Every Yee sample
 *    outside that range is a PEC-wall E sample or a wall-normal H sample that
 *    is identically zero.
 *  - A context is not thread safe; distinct contexts are independent.
 */
#ifndef YEE_H_
#define YEE_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define YEE_API_VERSION 1

typedef enum {
    YEE_OK = 0,
    YEE_EINVAL = -1,     /* invalid argument or configuration */
    YEE_ENOMEM = -2,     /* workspace too small */
    YEE_EHIP = -3,       /* a HIP runtime call failed */
    YEE_ESTATE = -4,     /* call not valid in the context's current state */
    YEE_ENUMERIC = -5,   /* non-finite value detected */
    YEE_EAGAIN = -6,     /* resource busy (serving: no slot or memory) */
    YEE_EOVERFLOW = -7   /* value outside the storage format's range */
} yee_status;

typedef enum {
    YEE_F64 = 0,         /* FP64 storage and arithmetic */
    YEE_F32 = 1,         /* FP32 storage and arithmetic */
    YEE_F16S = 2         /* FP16 storage x 2^s per component, FP32 arithmetic */
} yee_precision;

typedef enum { YEE_EX = 0, YEE_EY, YEE_EZ, YEE_HX, YEE_HY, YEE_HZ } yee_component;

typedef enum {
    YEE_GAUSS_DERIV = 0, /* w(t) = -2 u exp(-u^2),                    u = (t - t0)/tau */
    YEE_MOD_GAUSS = 1    /* w(t) = sin(2 pi f0 (t - t0)) exp(-u^2)                    */
} yee_waveform;

/* Grid description (Yee 1966 grid; CPML per Roden & Gedney 2000). */
typedef struct {
    int32_t nx, ny, nz;        /* cells; 2 <= n; nx <= 512 */
    double dx, dy, dz;         /* cell sizes in metres, > 0 */
    double courant;            /* S in (0, 1]: dt = S / (c0 sqrt(dx^-2 + dy^-2 + dz^-2)) */
    int32_t precision;         /* yee_precision */
    int32_t cpml_cells[3];     /* CPML thickness L per axis (both faces); 0 = bare PEC face;
                                  2 L <= n on that axis */
    double cpml_m;             /* grading order m >= 0 (sigma, kappa ~ x^m) */
    double cpml_sigma_max;     /* < 0: 0.8 (m + 1)/(eta0 dw) per axis; >= 0: used as given */
    double cpml_kappa_max;     /* >= 1 */
    double cpml_alpha_max;     /* >= 0 (S/m) */
    int32_t fp16_exp[6];       /* YEE_F16S: component c is stored as fp16(x * 2^fp16_exp[c]) */
    int32_t series_len;        /* probe samples kept per probe (ring of the last series_len
                                  steps); >= 1 */
} yee_grid_desc;

/* Soft point source (additive, not scaled by the update coefficient): after
 * the E half-update of step n (n = 0, 1, ...), the E sample (component, i, j, k)
 * gains amp * w((n + 1) dt).  Times in seconds, f0 in Hz, tau > 0. */
typedef struct {
    int32_t component;         /* YEE_EX, YEE_EY or YEE_EZ */
    int32_t i, j, k;
    int32_t waveform;          /* yee_waveform */
    double amp, t0, tau, f0;
} yee_source;

typedef struct yee_ctx yee_ctx;

/* Thread-local message describing the last failing call ("" if none). */
const char* yee_last_error(void);
int32_t yee_api_version(void);

/* Validate the description (sizes, Courant number, CPML thickness) and
 * create a context.  No device work.  *out is set to NULL on failure. */
yee_status yee_create(const yee_grid_desc* desc, yee_ctx** out);
void yee_destroy(yee_ctx* ctx);

/* The time step dt the context uses (seconds). */
yee_status yee_time_step(const yee_ctx* ctx, double* dt);

/* Materials on a rectilinear block lattice (Taflove & Hagness ch. 3 lossy
 * update).  seg_x[nx], seg_y[ny], seg_z[nz] give each cell's block index
 * along each axis (0 <= seg < ns*); eps_r and sigma (S/m) are indexed
 * [(bz * nsy + by) * nsx + bx], eps_r >= 1e-3, sigma >= 0.  The E samples of
 * cell (i, j, k) use that cell's block:
 *     Ca = (1 - s)/(1 + s),  Cb = (dt/(eps0 eps_r))/(1 + s),  s = sigma dt/(2 eps0 eps_r).
 * Before yee_bind_workspace() any lattice is accepted; afterwards only one
 * with the same (nsx, nsy, nsz) (it is re-uploaded by the next yee_reset()
 * or yee_upload_materials()).  Default: vacuum (one block, eps_r 1, sigma 0). */
yee_status yee_set_materials(yee_ctx* ctx, int32_t nsx, int32_t nsy, int32_t nsz,
                             const int32_t* seg_x, const int32_t* seg_y, const int32_t* seg_z,
                             const double* eps_r, const double* sigma);
/* Upload the current material table to the bound workspace (stream-ordered). */
yee_status yee_upload_materials(yee_ctx* ctx, void* stream);

/* PEC mask on the z-plane k (0 < k < nz): mask[j * nx + i] bit 0 holds Ex,
 * bit 1 Ey, bit 2 Ez of sample (i, j, k) at Ca = Cb = 0 (the sample stays 0).
 * A plane given again is merged (OR).  Only before yee_bind_workspace(). */
yee_status yee_add_pec_plane(yee_ctx* ctx, int32_t k, const uint8_t* mask);

/* Volume PEC mask: mask[(k * ny + j) * nx + i] bit 0 holds Ex, bit 1 Ey,
 * bit 2 Ez of sample (i, j, k) at Ca = Cb = 0 (the update leaves 0 there; a
 * source on the sample still adds after it), for every k in [0, nz)
 * (Ez of plane 0 lies inside the box; Ex and Ey of plane 0 are on the PEC
 * face anyway).  Other bits set: YEE_EINVAL.  The mask is merged (OR) with
 * plane masks of yee_add_pec_plane(); the device holds ny * nx bytes per
 * z-plane with a set bit and none for the others.  Only before
 * yee_bind_workspace(). */
yee_status yee_set_pec_mask(yee_ctx* ctx, const uint8_t* mask);

/* Soft source (see yee_source).  Only before yee_bind_workspace(). */
yee_status yee_add_source(yee_ctx* ctx, const yee_source* src);

/* Probe recording component `component` (0..5) at (i, j, k) after every
 * step: E^{n+1} for E components, H^{n+1/2} for H components, as stored (in
 * YEE_F16S: the decoded fp16 value).  *id receives the probe index.  Only
 * before yee_bind_workspace(). */
yee_status yee_add_probe(yee_ctx* ctx, int32_t component, int32_t i, int32_t j, int32_t k,
                         int32_t* id);

/* Frequencies (Hz) of the running DFT shared by all probes:
 * X_p(f) = sum_{n >= 1} y_p[n] exp(-i 2 pi f n dt) dt, accumulated in FP64.
 * Only before yee_bind_workspace(); nf may be 0. */
yee_status yee_set_dft_freqs(yee_ctx* ctx, const double* freqs, int32_t nf);

/* Device bytes one context needs for its current configuration. */
yee_status yee_footprint(const yee_ctx* ctx, int64_t* bytes);

/* Hand the caller-owned device buffer to the context (>= footprint bytes,
 * 256-byte aligned).  Freezes sources, probes, PEC planes and DFT
 * frequencies.  The buffer must outlive the context's use of it. */
yee_status yee_bind_workspace(yee_ctx* ctx, void* device_ptr, int64_t bytes);

/* Zero every field, CPML auxiliary, probe ring and DFT accumulator, set the
 * step counter to 0 and upload all tables.  Stream-ordered. */
yee_status yee_reset(yee_ctx* ctx, void* stream);

/* Overwrite one component (initial E^0 or H^{-1/2}) from host[nz][ny][nx].
 * Synchronizes the stream.  In YEE_F16S the values are rounded to storage;
 * a finite value with |x 2^fp16_exp| > 65504 returns YEE_EOVERFLOW and
 * nothing is written.  Non-finite values are stored as given (and reported
 * by yee_status_flags()). */
yee_status yee_set_field(yee_ctx* ctx, int32_t component, const double* host, void* stream);

/* Advance n_steps leapfrog steps (E^n, H^{n-1/2}) -> (E^{n+1}, H^{n+1/2}).
 * Asynchronous on `stream`; probe samples and DFT sums are folded on the
 * same stream. */
yee_status yee_step(yee_ctx* ctx, int64_t n_steps, void* stream);

/* Steps taken since the last yee_reset(). */
yee_status yee_steps_done(const yee_ctx* ctx, int64_t* n);

/* Copy one component to host[nz][ny][nx] (doubles).  Synchronizes. */
yee_status yee_read_field(yee_ctx* ctx, int32_t component, double* host, void* stream);

/* Probe samples y_p[n] for n = first .. first+count-1 (n = 1 is the value
 * after the first step) into host[count][n_probes].  The samples must still
 * be in the ring (the last series_len steps).  Synchronizes. */
yee_status yee_read_series(yee_ctx* ctx, int64_t first, int64_t count, double* host, void* stream);

/* DFT accumulators into re[n_probes][nf], im[n_probes][nf].  Synchronizes. */
yee_status yee_read_dft(yee_ctx* ctx, double* re, double* im, void* stream);

/* Health of the run: folds the probe samples not yet in the DFT, then scans
 * the current fields, the probe ring and the DFT accumulators, and writes the
 * context's sticky flags (cleared by yee_reset(), saved with the state):
 *   YEE_FLAG_NONFINITE  a NaN or infinity (FP16 storage: a NaN) is in the
 *                       fields, the probe ring or the DFT now, or was in a
 *                       probe sample folded into the DFT since the reset;
 *   YEE_FLAG_OVERFLOW   FP16 storage holds an infinity: some update produced
 *                       |x 2^fp16_exp| >= 65520, which rounds past the
 *                       largest finite fp16 (65504).
 * Returns YEE_EOVERFLOW if YEE_FLAG_OVERFLOW is set, else YEE_ENUMERIC if
 * YEE_FLAG_NONFINITE is set, else YEE_OK (flags are written in every case).
 * Reads the field set once (about the traffic of a third of a step);
 * synchronizes the stream. */
#define YEE_FLAG_NONFINITE 1u
#define YEE_FLAG_OVERFLOW 2u
yee_status yee_status_flags(yee_ctx* ctx, uint32_t* flags, void* stream);

/* Saved state (checkpoint/restart of a run): the current fields, CPML
 * auxiliaries, probe ring, DFT accumulators, status flags and the step and
 * fold counters, in one device buffer of yee_state_bytes() bytes (any
 * alignment) that the caller owns.  Materials, sources, probe positions and
 * frequencies are configuration, not state: a state loads into any bound
 * context of the same shape (grid, precision, CPML thickness, FP16
 * exponents, probe and frequency counts, ring length), which then continues
 * exactly as the saved one would have (fields and probe series bitwise; the
 * DFT sums in another order where the fold points differ).
 * yee_save_state: asynchronous on `stream` (a header kernel and device
 * copies); YEE_ENOMEM if bytes is too small.
 * yee_load_state: reads and checks the header (synchronizes the stream), then
 * queues the copies on `stream`; YEE_EINVAL for a buffer that is not a saved
 * state or is of another shape, YEE_ESTATE while the context is admitted to
 * a batch.  The source must stay valid until the stream passes the copies. */
yee_status yee_state_bytes(const yee_ctx* ctx, int64_t* bytes);
yee_status yee_save_state(yee_ctx* ctx, void* device_dst, int64_t bytes, void* stream);
yee_status yee_load_state(yee_ctx* ctx, const void* device_src, int64_t bytes, void* stream);

/* Port voltages and scattering parameters from two runs' probe DFTs (the
 * "S-parameter accumulators" are the running DFTs above; this combines them on
 * the host, in FP64, with no GPU work).  Port q is the probe list
 * port_probe[port_off[q] .. port_off[q+1]) with weights port_weight (a line
 * integral of E when the weights are cell lengths):
 *     V_q(f) = sum_i port_weight[i] X_{port_probe[i]}(f).
 * The two-run method (Sheen, Ali, Abouzahra and Kong, IEEE Trans. Microwave
 * Theory Tech. 38, 1990): the reference run (dft_ref: the uniform structure)
 * carries the incident wave, the device run (dft_dut) the total field; with
 * the source in front of port 0,
 *     S_00 = (V_0^dut - V_0^ref) / V_0^ref,   S_q0 = V_q^dut / V_q^ref (q > 0),
 * each referred to its own port position.
 *   dft_*_re/im  [n_probes][n_freq] host arrays, as yee_read_dft writes them.
 *   v_ref_re/im, v_dut_re/im  [n_ports][n_freq] outputs, or NULL.
 *   s_re, s_im   [n_ports][n_freq] outputs.
 * YEE_EINVAL for non-positive sizes, NULL required arrays, a non-increasing
 * port_off or a probe index outside [0, n_probes).  A zero reference voltage
 * gives IEEE infinities or NaNs in s. */
yee_status yee_sparams(int32_t n_probes, int32_t n_freq, const double* dft_ref_re, const double* dft_ref_im,
                       const double* dft_dut_re, const double* dft_dut_im, int32_t n_ports,
                       const int32_t* port_off, const int32_t* port_probe, const double* port_weight,
                       double* v_ref_re, double* v_ref_im, double* v_dut_re, double* v_dut_im, double* s_re,
                       double* s_im);

/* Launch shape of the fused step kernel: y-rows per workgroup tile, planes
 * per z-chunk and x samples per lane (1, 2 or 4); 0 keeps the automatic
 * choice (one sample per lane up to 256 samples per row, and in FP32 up to
 * 512; workgroups of at most 12 waves; the shortest chunk, at least 8 planes,
 * that lets every tile be resident on the device at once).  A workgroup holds
 * (tile_rows + 1) * ceil(nx / (64 * samples)) waves, at most 16.  Results do
 * not depend on the launch shape. */
yee_status yee_set_launch(yee_ctx* ctx, int32_t tile_rows, int32_t chunk_planes, int32_t samples_per_lane);

/* Steps per sweep of yee_step.  A two-step sweep reads the fields and CPML
 * auxiliaries once and writes them once for two leapfrog steps (time
 * blocking): each workgroup recomputes the first step on a halo of two rows
 * and two planes around its tile.  Every sample is computed by the same
 * instruction sequence as in a single step, so results are bitwise equal to
 * single steps.  steps_per_sweep: 0 automatic (two-step sweeps where they
 * apply: FP32 or FP16 storage, nx <= 256, a probe ring of at least 2 steps;
 * single steps otherwise and for the last step of an odd count), 1 single
 * steps only, 2 two-step sweeps (YEE_EINVAL where they do not apply).
 * tile_rows (1..9, the workgroup holds tile_rows + 3 waves) and
 * chunk_planes set the sweep's tile; 0 = automatic (9 rows, the shortest
 * chunk that lets every tile be resident at once). */
yee_status yee_set_time_blocking(yee_ctx* ctx, int32_t steps_per_sweep, int32_t tile_rows, int32_t chunk_planes);

/* The launch yee_step will use (after yee_bind_workspace): steps per sweep
 * (1 or 2), tile rows, planes per chunk and x samples per lane. */
yee_status yee_launch_info(const yee_ctx* ctx, int32_t* steps_per_sweep, int32_t* tile_rows, int32_t* chunk_planes,
                           int32_t* samples_per_lane);

/* Debug: tile-ownership check.  With a count buffer set, every single step
 * of yee_step (two-step sweeps are not taken meanwhile) adds one, with an
 * atomic, to the count of each element of the output field set it stores:
 * component c (0..5) of sample (i, j, k) at
 *     counts[c * comp_stride + (k * ny + j) * row_pitch + i].
 * After one step every stored sample (i < nx, j < ny, k < nz) must count
 * exactly one (it belongs to exactly one tile); padding columns i >= nx may
 * count one (vector stores of a lane's last samples, zeros), and the zero
 * plane k = nz none.  The caller owns the buffer (uint32, at least
 * 6 * comp_stride elements, zeroed by the caller); NULL switches counting
 * off.  Much slower than a plain step: for small test grids. */
yee_status yee_debug_layout(const yee_ctx* ctx, int64_t* comp_stride, int32_t* row_pitch);
yee_status yee_debug_set_write_counts(yee_ctx* ctx, uint32_t* device_counts, int64_t n_elems);

/* ------------------------------------------------------------------------
 * Batched stepper for serving many grids (continuous batching).
 *
 * One launch advances every admitted context ("slot") by one leapfrog step;
 * a replay is steps_per_replay such launches captured once in a HIP graph.
 * Requests are admitted and retired between replays, so requests that arrive
 * while others run join the next replay as slots and memory free up.  The
 * update of each grid is the same operation as yee_step() (results do not
 * depend on batching).  A batch takes contexts of one storage precision
 * (yee_batch_set_precision; FP32 unless set): FP32 and FP64 with nx <= 256,
 * FP16 storage with nx <= 512.  Contexts with probes need
 * series_len >= steps_per_replay.
 *
 * The caller owns the batch's device descriptor table (yee_batch_footprint()
 * bytes, handed over with yee_batch_bind_workspace()) as well as every
 * context's workspace; the admission budget counts context footprints.
 * ------------------------------------------------------------------------ */
typedef struct yee_batch yee_batch;

yee_status yee_batch_footprint(int32_t max_slots, int64_t* bytes);
/* hbm_budget: sum of admitted context footprints allowed at one time (bytes). */
yee_status yee_batch_create(int32_t max_slots, int64_t hbm_budget, int32_t steps_per_replay, yee_batch** out);
/* The storage precision (yee_precision) of the contexts the batch admits;
 * set before yee_batch_bind_workspace (YEE_ESTATE after it, YEE_EINVAL for an
 * unknown value).  The footprint does not depend on it. */
yee_status yee_batch_set_precision(yee_batch* batch, int32_t precision);
void yee_batch_destroy(yee_batch* batch);
yee_status yee_batch_bind_workspace(yee_batch* batch, void* device_ptr, int64_t bytes);
/* Admit a bound context for n_steps more steps.  YEE_EAGAIN: no free slot or
 * the footprint would exceed the budget (nothing changes; retry later). */
yee_status yee_batch_admit(yee_batch* batch, yee_ctx* ctx, int64_t n_steps, int32_t* slot);
/* One replay (steps_per_replay steps of every admitted, unfinished slot),
 * queued on `stream` without waiting for earlier replays (the descriptor
 * table is rewritten by a copy on the same stream, behind them): successive
 * runs of one batch must use one stream.  Probe DFTs are folded after it. */
yee_status yee_batch_run(yee_batch* batch, void* stream);
/* yee_step may also advance an admitted context between replays, on the
 * batch's stream (for instance a lone request in its own launch shape): the
 * next replay continues from the context's current step. */
/* Slots whose requested steps are all taken (up to cap written to done). */
yee_status yee_batch_poll(yee_batch* batch, int32_t* done, int32_t cap, int32_t* n_done);
/* Retire a slot (its context stays valid; read results before or after). */
yee_status yee_batch_release(yee_batch* batch, int32_t slot);
yee_status yee_batch_info(const yee_batch* batch, int32_t* active_slots, int64_t* bytes_in_use);

/* ------------------------------------------------------------------------
 * Discrete adjoint: gradient of a probe objective with respect to eps_r.
 *
 * Objective  J = sum_{n=1}^{N} sum_p y_p[n]^2  over every probe of the
 * context (y_p[n] as recorded by yee_add_probe; a sample probed twice counts
 * twice).  Gradient  g(i, j, k) = dJ / d eps_r(i, j, k)  for each cell of a box
 * [i0, i1) x [j0, j1) x [k0, k1), where eps_r of a cell enters only through
 * Ca and Cb of the cell's three E samples (the materials formula of
 * yee_set_materials; E samples on the outer faces or under a PEC mask do not
 * depend on it).  The gradient is the exact derivative of the discrete update
 * (reverse-mode: the transposed step applied backward in time, Giles & Pierce
 * 2000 on discrete adjoints; CPML recursions included), not of the continuous
 * equations.  The paper defines no solver and no adjoint.
 *
 * Schedule: yee_adjoint_forward() runs the N steps from step 0, storing
 * (E, H, psi) every checkpoint_every steps and the probe samples of every step;
 * yee_adjoint_backward() walks the segments newest first, restores each
 * checkpoint, recomputes its steps (storing E of the box cells) and runs the
 * reverse steps.  Adjoint fields use the context's compute precision; the
 * gradient is accumulated in FP64.  Contexts must be YEE_F64 or YEE_F32.
 *
 * The caller owns the adjoint's device workspace (yee_adjoint_footprint()
 * bytes, 256-byte aligned): (N/K + 1) checkpoints of the context state,
 * K + 1 copies of E over the box per kept history segment (one unless
 * yee_adjoint_set_history() asks for more), 12 adjoint arrays of the grid's
 * size and N x n_probes doubles.
 * ------------------------------------------------------------------------ */
typedef struct yee_adjoint yee_adjoint;

/* box = {i0, i1, j0, j1, k0, k1} with 0 <= lo < hi <= n per axis.  The context
 * must be bound; its probes and grid fix the workspace size. */
yee_status yee_adjoint_create(yee_ctx* ctx, int64_t n_steps, int32_t checkpoint_every,
                              const int32_t* box, yee_adjoint** out);
void yee_adjoint_destroy(yee_adjoint* adj);

/* How many segments (the newest) keep the E history of the box from the
 * forward run: 1 by default, the checkpoint-recompute schedule above; 0 keeps
 * all of them, and the backward run then recomputes nothing.  Every kept
 * segment adds (K + 1) x 3 x box cells x element bytes to the workspace (FP32
 * 128^3 with a 64^3 box and K = 64: 204 MB per segment, 3.3 GB for 16).  The
 * gradient does not depend on it: recomputed and kept histories are the same
 * values.  Call before yee_adjoint_footprint(); YEE_ESTATE once bound,
 * YEE_EINVAL outside [0, number of segments]. */
yee_status yee_adjoint_set_history(yee_adjoint* adj, int32_t segments);
yee_status yee_adjoint_footprint(const yee_adjoint* adj, int64_t* bytes);
yee_status yee_adjoint_bind_workspace(yee_adjoint* adj, void* device_ptr, int64_t bytes);

/* Forward run of n_steps from the context's state at step 0 (after
 * yee_reset() and optional yee_set_field(); materials uploaded and unchanged
 * until the backward run ends).  Leaves the context exactly as yee_step()
 * would (fields, probe ring, DFT) and writes J to *objective (host).
 * Synchronizes the stream.  YEE_ESTATE if the context is not at step 0. */
yee_status yee_adjoint_forward(yee_adjoint* adj, double* objective, void* stream);

/* Gradient of the last forward run into grad (device pointer, FP64,
 * [k1-k0][j1-j0][i1-i0], i fastest; overwritten).  Asynchronous on `stream`;
 * the context returns to its state after the forward run.  YEE_ESTATE if no
 * forward run was recorded or the context was stepped since. */
yee_status yee_adjoint_backward(yee_adjoint* adj, double* grad, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* YEE_H_ */
