/* raymeta.h -- C ABI of libraymeta: radar IF synthesis from ray meta data on
 * one MI355X (gfx950).
 *
 * The operation is the method of Section II of the paper: a ray tracer has
 * stored, per ray, the ordered list of triangles it hit (mesh ID a_k,
 * triangle index b_k, barycentric coordinates u_k, v_k; Section II.B).  For
 * each chirp j the hit points are moved with the animated vertices (Eq. 6),
 * the path length TX -> hits -> RX is formed for each antenna pair (Section
 * II.A; Eq. 7 for displaced antennas), converted to a delay (Eq. 1) and
 * summed into the FMCW beat signal (Eq. 2, slope mu = B / T_c of Eq. 3):
 *
 *     s_q(t_n, j) = sum_i w_i exp(2 pi i (mu t_n tau_i + f_c tau_i)),
 *     t_n = n / f_s,  n = 0 .. n_samples - 1,
 *
 * with w_i the per-ray weight (pattern A times an Eq. 5 span mask).  The
 * range-Doppler map is the 2-D DFT of each pair's [chirp][sample] block
 * (Eq. 4).
 *
 * Conventions.
 *   - All array arguments are DEVICE pointers owned by the caller (allocated
 *     for example with torch); the library allocates nothing and keeps no
 *     state between calls.  Scalars and the small descriptor structs are read
 *     by value during the call.
 *   - Every call is asynchronous on the given stream (0 = the null stream)
 *     unless it says otherwise; inputs must stay valid until the stream has
 *     run the work.
 *   - Every call returns an rmd_status and, on failure, leaves a message in
 *     rmd_last_error() (thread-local).  Argument errors (RMD_EINVAL) are found
 *     before anything is launched; RMD_EHIP from rmd_if_cube can follow
 *     launches of earlier chirp batches already queued on the stream.
 *   - Complex values are interleaved float pairs (re, im).
 */
#ifndef RAYMETA_H
#define RAYMETA_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rmd_status;
#define RMD_OK       0
#define RMD_EINVAL  (-1)   /* bad argument, size or pointer */
#define RMD_EHIP    (-3)   /* a HIP call failed */
#define RMD_ESCENE  (-8)   /* rmd_check_scene found out-of-range meta data */

#define RMD_MAX_SAMPLES 1024   /* n_samples limit of rmd_if_cube */
#define RMD_MAX_FFT     4096   /* line length limit of rmd_range_doppler */
#define RMD_MAX_RAYS    (1 << 30)   /* n_rays limit (32-bit ray indices with partition headroom) */

/* FMCW parameters (Section II.A, Eq. 3). */
typedef struct {
    double  f_c;         /* carrier frequency [Hz] */
    double  bandwidth;   /* sweep bandwidth B [Hz] */
    double  t_chirp;     /* chirp duration T_c [s]; mu = B / T_c */
    double  f_s;         /* IF sampling rate [Hz]; t_n = n / f_s */
    int32_t n_samples;   /* samples per chirp, 1 .. RMD_MAX_SAMPLES */
    int32_t n_chirps;    /* chirps (vertex snapshots) in the scene */
} rmd_radar;

/* Scene and ray meta data (Section II.B), all device arrays.
 *   mesh_tri_off [n_meshes + 1]  triangles of mesh a are [off[a], off[a+1])
 *   tris         [n_tris][3]     global vertex indices of each triangle
 *   verts        [n_chirps][n_verts][3] float64 vertex positions of the
 *                                snapshot taken for chirp j (metres)
 *   ray_off      [n_rays + 1]    hits of ray i are [ray_off[i], ray_off[i+1]),
 *                                first hit first
 *   hit_mesh, hit_tri [n_hits]   a_k and b_k (b_k counts within mesh a_k)
 *   hit_u, hit_v      [n_hits]   barycentric coordinates (float32)
 * A ray with no hits, or whose meta data is out of range (an offset outside
 * [0, n_hits], a mesh, triangle or vertex index outside its array),
 * contributes nothing: the kernels check every index before using it, so
 * bad meta data never causes an out-of-bounds access.  rmd_check_scene
 * reports such entries. */
typedef struct {
    int32_t n_meshes, n_tris, n_verts, n_rays;
    int64_t n_hits;
    const int32_t* mesh_tri_off;
    const int32_t* tris;
    const double*  verts;
    const int32_t* ray_off;
    const int32_t* hit_mesh;
    const int32_t* hit_tri;
    const float*   hit_u;
    const float*   hit_v;
} rmd_scene;

int32_t     rmd_api_version(void);
const char* rmd_last_error(void);

/* Counts rays whose meta data is out of range (see rmd_scene) into
 * *n_bad_rays.  Synchronous: waits for the stream.  Returns RMD_ESCENE when
 * the count is not zero.  `workspace` needs 8 bytes. */
rmd_status rmd_check_scene(const rmd_scene* scene, int32_t n_chirps, void* workspace,
                           int64_t* n_bad_rays, hipStream_t stream);

/* Bytes of device workspace rmd_if_cube and rmd_if_cube_direct need for these
 * sizes (one size serves both).  Chirps are processed in batches of up to 16
 * whose per-ray geometry (7 float64 per ray and chirp: inner path length,
 * first and last hit point) fits in 1 GiB; the workspace holds the geometry
 * of one batch, or of two when there are several (the next batch's geometry
 * is built on a library-owned helper stream of the device while the current
 * batch is synthesised; events join it back into the caller's stream),
 * every hit resolved to its triangle's vertex indices and
 * barycentric coordinates (20 bytes per hit, once per call), and the batch's
 * per-partition results (rmd_if_cube: a grid of M
 * complex64 cells per ray partition, pair and chirp, M the smallest power of
 * two >= max(64, 2 n_samples), plus n_samples float64; rmd_if_cube_direct:
 * n_samples complex64 per ray partition, pair and chirp). */
rmd_status rmd_workspace_bytes(const rmd_scene* scene, const rmd_radar* radar, int32_t n_pairs,
                               int32_t chirp_count, int64_t* bytes);

/* IF cube, Eqs. 1, 2, 3, 6, 7 (Section II.A, II.D, II.E).
 *   pairs    [n_pairs][6] float64: displaced TX position x'_tx then RX
 *            position x'_rx of each antenna pair (Eq. 7).  The path length of
 *            pair q is the inner path (first hit -> last hit) plus
 *            |p^f - x'_tx| + |p^l - x'_rx|, which is Eq. 7 with the traced
 *            pair's legs cancelled exactly.
 *   weights  [n_rays] float32 per-ray weight w_i, or NULL for w_i = 1.
 *   chirps   [chirp0, chirp0 + chirp_count) of the scene's n_chirps.
 *   s        output [n_pairs][chirp_count][n_samples] complex64.
 *   workspace at least rmd_workspace_bytes(...) bytes, 256-byte aligned.
 * The sum over rays is evaluated as a type-1 non-uniform FFT: each ray's
 * phasor (phase formed in float64 and reduced modulo one cycle) is spread
 * onto a 2x-oversampled periodic grid with an 8-cell "exponential of
 * semicircle" kernel, the grid is transformed and deconvolved in float64.
 * The grid accumulates 64-bit fixed-point integers scaled by the largest
 * |w_i| (each contribution cut toward zero by less than 2^-29 max|w|), so its sums are
 * exact and order-free, and partition grids are added in float64 in a fixed
 * order: repeated calls give identical results.  The kernel's aliasing error
 * is about 1e-7 relative; with the float32 phasors the result agrees with
 * the exact sum to about 1e-6 (relative L2 per pair and chirp).  Weights must
 * be finite. */
rmd_status rmd_if_cube(const rmd_scene* scene, const rmd_radar* radar, int32_t n_pairs, const double* pairs,
                       const float* weights, int32_t chirp0, int32_t chirp_count, float* s,
                       void* workspace, int64_t workspace_bytes, hipStream_t stream);

/* The IF cube of rmd_if_cube (same arguments, checks, method and output,
 * bitwise) for callers that cannot allocate device memory: code being
 * captured into a HIP graph, allocation-free serving loops, harnesses that
 * forbid hipMalloc.  The workspace is a static device array of
 * RMD_STATIC_SCRATCH_BYTES that each GPU holds from the library's first use
 * until the process ends; nothing is allocated or freed per call.  Sizes
 * whose rmd_workspace_bytes() exceeds it return RMD_EINVAL (use rmd_if_cube
 * with a caller workspace).  Every call on one GPU shares that GPU's array,
 * so calls that overlap in time on one GPU (different streams, or different
 * threads without ordering) race and give wrong results; calls queued on one
 * stream are ordered and safe.  Nothing in the array has to start at zero
 * (every word a call reads it first writes).  The first call on each device
 * looks up the array's device address (hipGetSymbolAddress); make it outside
 * graph capture. */
#define RMD_STATIC_SCRATCH_BYTES (64ll << 20)
rmd_status rmd_if_cube_static(const rmd_scene* scene, const rmd_radar* radar, int32_t n_pairs, const double* pairs,
                              const float* weights, int32_t chirp0, int32_t chirp_count, float* s,
                              hipStream_t stream);

/* The same IF cube with the sum over rays evaluated term by term: the arguments,
 * checks and output are those of rmd_if_cube.  Phases are formed in float64 and
 * reduced modulo one cycle; the phasors are float32, split into fp16 high and
 * low parts for the matrix products (float32 accumulation, about 2^-21
 * relative); partition sums are added in float64 in a fixed order, so repeated
 * calls give identical results.  Slower than rmd_if_cube; exact up to
 * rounding. */
rmd_status rmd_if_cube_direct(const rmd_scene* scene, const rmd_radar* radar, int32_t n_pairs,
                              const double* pairs, const float* weights, int32_t chirp0, int32_t chirp_count,
                              float* s, void* workspace, int64_t workspace_bytes, hipStream_t stream);

/* Range-Doppler map, Eq. 4: S[q] = DFT_2d(s[q]) over (chirp, sample), the
 * forward unnormalised transform exp(-2 pi i k n / N) on both axes, without
 * window or padding.  s and S are [n_pairs][n_chirps][n_samples] complex64;
 * S may equal s (in place).  n_chirps and n_samples must be powers of two
 * no larger than RMD_MAX_FFT. */
rmd_status rmd_range_doppler(const float* s, float* S, int32_t n_pairs, int32_t n_chirps, int32_t n_samples,
                             hipStream_t stream);

/* Eq. 5 span rule (Section II.C): a ray is kept when
 *   mode 0 (ANY):  at least one hit is on a mesh of the set,
 *   mode 1 (NONE): no hit is on a mesh of the set,
 *   mode 2 (ALL):  every hit is on a mesh of the set,
 * and its hit count lies in [min_hits, max_hits]. */
typedef struct {
    int32_t mode;
    int32_t min_hits;
    int32_t max_hits;
} rmd_span_rule;

/* weights[i] = (amp ? amp[i] : 1) if ray i is kept by the rule, else 0.
 *   in_set  [n_meshes] uint8: nonzero for the meshes of the rule's set.
 *   amp     [n_rays] float32 or NULL.  weights [n_rays] float32 output. */
rmd_status rmd_span_weights(const rmd_scene* scene, const uint8_t* in_set, const rmd_span_rule* rule,
                            const float* amp, float* weights, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* RAYMETA_H */
