// libraymeta: radar IF synthesis from ray meta data (Section II, Eqs. 1-7)
// for gfx950.  The C ABI is declared in include/raymeta.h.
//
// Kernels:
//   resolve_kernel each hit's triangle and vertex indices range-checked and
//                  reduced to a record, once per call.
//   geometry_kernel Eq. 6 for every hit of a ray and the pair-independent
//                  part of its path (FP64), once per ray and chirp.
//   spread_kernel  Eqs. 7, 1, 2 (rmd_if_cube): per workgroup one antenna pair,
//                  one chirp and one partition of the rays; the antenna legs
//                  and phases per ray in FP64, then each ray's phasor spread
//                  onto an oversampled periodic grid in LDS (the sum over rays
//                  as a type-1 non-uniform FFT), in 64-bit fixed point.
//   wmax_kernel    the largest weight (sets the fixed-point scale).
//   deconv_kernel  the spreading kernel's Fourier transform at the output
//                  frequencies (FP64 quadrature), once per call.
//   finish_kernel  per (pair, chirp): the partitions' grids summed in FP64,
//                  their inverse DFT (FP64, LDS) and the deconvolved samples.
//   synth_kernel   the same sum evaluated directly (rmd_if_cube_direct): MFMA
//                  products of phasor tiles split into fp16 high and low parts
//                  (fast time factored into 32 rows x 16 columns).
//   reduce_kernel  sums synth_kernel's partition cubes in FP64, fixed order.
//   fft_kernel     radix-2 FFT of lines held in LDS (Eq. 4, one axis a pass).
//   span_kernel    Eq. 5 rule masks, one thread per ray.
//   check_kernel   counts rays with out-of-range meta data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>

#include "raymeta.h"

namespace rmd {

constexpr int kWave = 64;
constexpr int kWaves = 4;                 // waves per synthesis workgroup
constexpr int kThreads = kWave * kWaves;
constexpr int kRows = 32;                 // MFMA tile rows m: fast-time steps of kCols samples
constexpr int kCols = 16;                 // MFMA tile columns k: consecutive samples
constexpr int kBlock = kRows * kCols;     // samples of one pass (512)
constexpr int kGroup = 16;                // rays per operand table (two MFMA blocks of 8)
constexpr int kBlockRays = 8;             // rays per 32 x 32 x 16 fp16 MFMA (K = 2 components x 8 rays)
constexpr int kSlotWords = 4;             // one lane's operand: 8 fp16 values
// Word offset of lane slot L in an operand block.  Slots are permuted within
// each run of 8 (XOR with the run index) so that the build's scattered 4-byte
// writes spread over the LDS banks; the block needs no padding.
__host__ __device__ constexpr int slot_word(int L) { return kSlotWords * (L ^ ((L >> 3) & 7)); }
constexpr int kBlockWords = kSlotWords * kWave;             // 256 words per block
constexpr int kArrayWords = (kGroup / kBlockRays) * kBlockWords;
constexpr int kTableWords = 4 * kArrayWords;                // A hi, A lo, B hi, B lo
static_assert(kWaves * kTableWords >= kWaves * 2 * kBlock, "wave sums must fit in the table memory");
static_assert(kRows / (kWave / kGroup) == 8 && kCols / (kWave / kGroup) == 4,
              "the build's step trees are written for 8 rows and 4 columns per lane");

typedef __fp16 f16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr double kC0 = 299792458.0;

// Spreading method.  The sum s[n] = sum_i c_i e^{2 pi i n theta_i}, n < N, is
// a Fourier series at N integer frequencies with non-uniform positions
// theta_i (cycles per sample, modulo 1).  With the centre index n_c = N / 2,
//   s[n_c + m] = sum_i c'_i e^{2 pi i m theta_i},  c'_i = c_i e^{2 pi i n_c theta_i},
// for m in [-N/2, N/2).  Each c'_i is spread onto a periodic grid of M >= 2N
// cells around x_i = M theta_i with a kernel psi of kTaps cells; the grid's
// inverse DFT G[m] = sum_l g[l] e^{2 pi i m l / M} then equals
// psi_hat(m / M) s[n_c + m] up to the kernel's aliasing error, psi_hat being
// the continuous Fourier transform of psi (Poisson summation).  psi is the
// "exponential of semicircle" kernel e^{beta (sqrt(1 - z^2) - 1)}, z = 2 u /
// kTaps for an offset of u cells (Barnett, Magland and af Klinteberg, SIAM J.
// Sci. Comput. 41, 2019): at 2x oversampling and 8 cells its aliasing error
// is about 1e-7 relative.  Kernel values are evaluated as one polynomial per
// tap (degree kTapDeg, fitted on the host), which keeps their float32 error at
// a few ulp; exp() of a float32 argument near -beta would lose about 1e-6.
// Degree 8 interpolates the kernel at Chebyshev points to 7e-9 of its peak
// (degree 10: 5e-9), both below float32's spacing there (6e-8), with 8 fewer
// multiply-adds per ray and pair.
constexpr int kTaps = 8;
constexpr int kTapDeg = 8;
static_assert(kTapDeg % 2 == 0 && kTaps % 2 == 0, "taps come in mirrored pairs; even degree");
constexpr double kBeta = 2.30 * kTaps;
constexpr int kMinGridLog2 = 6;          // M >= 64
constexpr int kGridCopies = 2;           // spreading grids per workgroup (lanes split by parity)
constexpr int kQuad = 256;               // trapezoid intervals of the psi_hat quadrature

struct SynthArgs {
    const int32_t* mesh_tri_off;
    const int32_t* tris;
    const double* verts;
    const int32_t* ray_off;
    const int32_t* hit_mesh;
    const int32_t* hit_tri;
    const float* hit_u;
    const float* hit_v;
    const double* pairs;
    const float* weights;
    double* geo;                // [7][chirp_count][n_rays]: inner path, first hit xyz, last hit xyz
    int4* hit_rec;              // [n_hits]: vertex indices i1, i2, i3 and the bits of u (i1 < 0: bad hit)
    float* hit_rec_v;           // [n_hits]: v
    float2* partial;            // [n_parts][n_pairs][chirp_count][n_samples]
    int64_t n_hits;
    int32_t n_meshes, n_tris, n_verts, n_rays;
    int32_t n_pairs, chirp0, chirp_count, n_samples;   // chirps [chirp0, chirp0 + chirp_count) of one batch
    int32_t n_parts, rays_per_part, n_passes;
    double cyc_per_m;           // f_c / c: carrier cycles per metre of path (Eq. 1 into Eq. 2)
    double step_per_m;          // mu / (c f_s): beat cycles per sample per metre (Eqs. 1-3)
    // spreading method: partial holds [n_parts][n_pairs][chirp_count][M] grids
    const double* deconv;       // [n_samples]: 1 / psi_hat((n - center) / M)
    const unsigned* wmax_bits;  // max_i |w_i| as float bits (1 when weights is NULL)
    int32_t grid_log2, center;  // M = 2^grid_log2; center n_c = n_samples / 2
    // Tap t < kTaps / 2 has the polynomial P_t(s) = E_t(s^2) + s O_t(s^2), s in
    // [-1/2, 1/2); psi is even, so tap kTaps - 1 - t is P_t(-s) = E_t - s O_t.
    float tap_even[kTaps / 2][kTapDeg / 2 + 1];   // E_t coefficients, constant term first
    float tap_odd[kTaps / 2][kTapDeg / 2];        // O_t coefficients
};

// sqrt(x) for finite x >= 0 from the hardware reciprocal square root: one
// Newton step on y = 1/sqrt(x), then one correction of the root s = x y,
// s + (y / 2)(x - s^2) (Markstein's method): each step doubles the correct
// bits, so from the instruction's 2^-20 or better the result is within a few
// ulp, against about 25 instructions for a correctly rounded root.  The
// antenna legs (tens of metres at 257 carrier cycles per metre) need about
// 1e-13 relative, and so do the inner paths.  x = 0 gives 0.
__device__ inline double sqrt_leg(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double hy = 0.5 * y;
    y = fma(hy, fma(-x, y * y, 1.0), y);
    const double sr = x * y;
    const double r = fma(-sr, sr, x);
    const double out = fma(0.5 * y, r, sr);
    return x == 0.0 ? 0.0 : out;
}

__device__ inline double leg3(double ax, double ay, double az, double bx, double by, double bz) {
    const double dx = ax - bx, dy = ay - by, dz = az - bz;
    return sqrt_leg(dx * dx + dy * dy + dz * dz);
}

// Eq. 6 for hit k on the snapshot `v` (n_verts x 3); false if any index of
// the hit is out of range.
__device__ inline bool hit_point(const SynthArgs& a, const double* __restrict__ v, int64_t k,
                                 double& px, double& py, double& pz) {
    const int32_t m = a.hit_mesh[k];
    if (m < 0 || m >= a.n_meshes) return false;
    const int32_t t0 = a.mesh_tri_off[m], t1 = a.mesh_tri_off[m + 1];
    const int32_t b = a.hit_tri[k];
    if (b < 0 || t0 < 0 || t1 > a.n_tris || b >= t1 - t0) return false;
    const int32_t t = t0 + b;
    const int32_t i1 = a.tris[3 * t], i2 = a.tris[3 * t + 1], i3 = a.tris[3 * t + 2];
    if ((unsigned)i1 >= (unsigned)a.n_verts || (unsigned)i2 >= (unsigned)a.n_verts ||
        (unsigned)i3 >= (unsigned)a.n_verts)
        return false;
    const double u = a.hit_u[k], w = a.hit_v[k];
    const double g = 1.0 - u - w;
    const double* v1 = v + 3 * (int64_t)i1;
    const double* v2 = v + 3 * (int64_t)i2;
    const double* v3 = v + 3 * (int64_t)i3;
    px = g * v1[0] + u * v2[0] + w * v3[0];
    py = g * v1[1] + u * v2[1] + w * v3[1];
    pz = g * v1[2] + u * v2[2] + w * v3[2];
    return true;
}

// Each hit resolved once per call: the vertex indices of its triangle and its
// barycentric coordinates, or i1 = -1 if any index of the hit is out of range.
__global__ void resolve_kernel(SynthArgs a) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= a.n_hits) return;
    int4 r = make_int4(-1, 0, 0, 0);
    const int32_t m = a.hit_mesh[k];
    if (m >= 0 && m < a.n_meshes) {
        const int32_t t0 = a.mesh_tri_off[m], t1 = a.mesh_tri_off[m + 1];
        const int32_t b = a.hit_tri[k];
        if (b >= 0 && t0 >= 0 && t1 <= a.n_tris && b < t1 - t0) {
            const int32_t t = t0 + b;
            const int32_t i1 = a.tris[3 * t], i2 = a.tris[3 * t + 1], i3 = a.tris[3 * t + 2];
            if ((unsigned)i1 < (unsigned)a.n_verts && (unsigned)i2 < (unsigned)a.n_verts &&
                (unsigned)i3 < (unsigned)a.n_verts)
                r = make_int4(i1, i2, i3, __float_as_int(a.hit_u[k]));
        }
    }
    a.hit_rec[k] = r;
    a.hit_rec_v[k] = a.hit_v[k];
}

// Eq. 6 for a resolved hit on the snapshot `v`.
__device__ inline void rec_point(const int4 r, float hv, const double* __restrict__ v, double& px, double& py,
                                 double& pz) {
    const double u = __int_as_float(r.w), w = hv;
    const double g = 1.0 - u - w;
    const double* v1 = v + 3 * (int64_t)r.x;
    const double* v2 = v + 3 * (int64_t)r.y;
    const double* v3 = v + 3 * (int64_t)r.z;
    px = g * v1[0] + u * v2[0] + w * v3[0];
    py = g * v1[1] + u * v2[1] + w * v3[1];
    pz = g * v1[2] + u * v2[2] + w * v3[2];
}

// The part of ray i's path that does not depend on the antenna pair, on the
// snapshot of chirp chirp0 + jj (Eq. 6 for every hit): the inner length from
// the first to the last hit and those two hit points.  One thread per (ray,
// chirp).  The hits' records are loaded kHitRun at a time before any vertex,
// so the common rays (up to kHitRun hits) wait for two dependent loads, not
// for one chain per hit.  The pair loop of the synthesis then only adds the
// two antenna legs.  A ray with no usable path (no hits, or out-of-range meta
// data) stores an inner length of -1.
constexpr int kHitRun = 4;

__global__ void geometry_kernel(SynthArgs a) {
    const int ray = blockIdx.x * blockDim.x + threadIdx.x;
    const int jj = blockIdx.y;
    if (ray >= a.n_rays) return;
    const int64_t plane = (int64_t)a.chirp_count * a.n_rays;
    double* g = a.geo + (int64_t)jj * a.n_rays + ray;
    const int32_t b = a.ray_off[ray], e = a.ray_off[ray + 1];
    const double* v = a.verts + (int64_t)(a.chirp0 + jj) * a.n_verts * 3;
    double fx = 0, fy = 0, fz = 0, lx = 0, ly = 0, lz = 0, inner = -1.0;
    if (b >= 0 && e <= a.n_hits && e > b) {
        inner = 0.0;
        for (int64_t k0 = b; k0 < e && inner >= 0.0; k0 += kHitRun) {
            int4 r[kHitRun];
            float hv[kHitRun];
#pragma unroll
            for (int c = 0; c < kHitRun; ++c) {
                r[c] = make_int4(0, 0, 0, 0);
                hv[c] = 0.0f;
                if (k0 + c < e) {
                    r[c] = a.hit_rec[k0 + c];
                    hv[c] = a.hit_rec_v[k0 + c];
                }
            }
#pragma unroll
            for (int c = 0; c < kHitRun; ++c) {
                if (k0 + c >= e) break;
                if (r[c].x < 0) {
                    inner = -1.0;
                    break;
                }
                double x, y, z;
                rec_point(r[c], hv[c], v, x, y, z);
                if (k0 + c == b) {
                    fx = x; fy = y; fz = z;
                } else {
                    inner += leg3(x, y, z, lx, ly, lz);
                }
                lx = x; ly = y; lz = z;
            }
        }
        if (inner < 0.0) fx = fy = fz = lx = ly = lz = 0.0;
    }
    g[0] = inner;
    g[plane] = fx;
    g[2 * plane] = fy;
    g[3 * plane] = fz;
    g[4 * plane] = lx;
    g[5 * plane] = ly;
    g[6 * plane] = lz;
}

// Pair-independent geometry of one ray on one batch chirp (see
// geometry_kernel) and its weight; w = 0 marks a ray that contributes nothing
// (outside the partition, or without a usable path).
struct Geo {
    double inner, fx, fy, fz, lx, ly, lz;
    float w;
};

__device__ inline Geo load_geo(const SynthArgs& a, int ray, int r1, int jj) {
    Geo g{0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0f};
    if (ray >= r1) return g;
    const int64_t plane = (int64_t)a.chirp_count * a.n_rays;
    const double* p = a.geo + (int64_t)jj * a.n_rays + ray;
    g.inner = p[0];
    g.fx = p[plane];
    g.fy = p[2 * plane];
    g.fz = p[3 * plane];
    g.lx = p[4 * plane];
    g.ly = p[5 * plane];
    g.lz = p[6 * plane];
    g.w = a.weights ? a.weights[ray] : 1.0f;
    return g;
}

// Phases of a ray for pair pq, in cycles modulo 1: the path length is the
// inner path plus |p^f - x'_tx| + |p^l - x'_rx| (Eq. 7 with the traced pair's
// legs cancelled exactly); Eq. 1 turns it into the delay, Eq. 2 into
// phi = f_c tau and theta = mu tau / f_s (the phase step per sample).
struct Phases {
    double phi, theta;
    float w;
};

__device__ inline Phases ray_phases(const SynthArgs& a, const Geo& g, const double* __restrict__ pq) {
    Phases p{0.0, 0.0, 0.0f};
    if (!(g.inner >= 0.0) || g.w == 0.0f) return p;
    const double len = g.inner + leg3(g.fx, g.fy, g.fz, pq[0], pq[1], pq[2]) +
                       leg3(g.lx, g.ly, g.lz, pq[3], pq[4], pq[5]);
    const double ph = len * a.cyc_per_m;              // f_c tau
    const double th = len * a.step_per_m;             // mu tau / f_s
    p.phi = ph - floor(ph);
    p.theta = th - floor(th);
    p.w = g.w;
    return p;
}

__device__ inline double frac1(double x) { return x - floor(x); }

// e^{2 pi i x} for x in [0, 1) revolutions, hardware sine and cosine.
__device__ inline float2 cis(double x) {
    const float xf = (float)x;
    return make_float2(__builtin_amdgcn_cosf(xf), __builtin_amdgcn_sinf(xf));
}

__device__ inline float2 cmul(float2 p, float2 z) {
    return make_float2(fmaf(p.x, z.x, -p.y * z.y), fmaf(p.x, z.y, p.y * z.x));
}

// Split two float32 values into fp16 high parts (rounded toward zero) and
// fp16 low parts (the rounded remainders): x = hi + lo to about 2^-21 |x|.
// Returns the packed pairs (x in the low half, y in the high half).
__device__ inline void split2(float x, float y, uint32_t& hi, uint32_t& lo) {
    const f16x2 h = __builtin_amdgcn_cvt_pkrtz(x, y);
    const f16x2 l = __builtin_amdgcn_cvt_pkrtz(fmaf((float)h.x, -1.0f, x), fmaf((float)h.y, -1.0f, y));
    hi = __builtin_bit_cast(uint32_t, h);
    lo = __builtin_bit_cast(uint32_t, l);
}

// Workgroup (pair q, pass b, partition p, chirp j).  Fast time is split as
// n = 512 b + 16 m + k (pass b, row m < 32, column k < 16), so that
//   s[n] = sum_i A[m][i] B[i][k],  A[m][i] = w_i e^{2 pi i (phi_i + (32 b + m) 16 theta_i)},
//                                 B[i][k] = e^{2 pi i k theta_i}:
// a complex 32 x 16 product over the rays, in real form a 32 x 32 product
// with two K entries per ray: A' = (Re A, Im A) and B' = ([Re B | Im B],
// [-Im B | Re B]), which puts Re s in result columns 0-15 and Im s in
// columns 16-31.
//
// The product runs on the fp16 matrix path: every operand value is split into
// fp16 high and low parts (split2), and A'B' is formed as hi hi + hi lo + lo hi
// with float32 accumulation (the dropped lo lo term is below 2^-21 of the
// product).  One 32 x 32 x 16 MFMA takes 8 rays (K = 2 components x 8); its
// operand layout puts A'[m][kk] in lane m + 32 (kk / 8), element kk % 8, and
// B'[kk][col] in lane col + 32 (kk / 8), element kk % 8, with kk = 2 r + c for
// ray r of the block and component c.
//
// Each wave takes the partition's rays 64 at a time (one ray per lane;
// super-groups round-robin over the waves):
//   phases  lane l derives ray l's phases in FP64 (antenna legs, Eq. 1, the
//           reductions modulo one cycle) and the float32 phasor steps between
//           rows and columns;
// then, for each group of kGroup = 16 of these rays,
//   build   the four lanes r, r + 16, r + 32, r + 48 fetch ray r's phases
//           from its owner lane (cross-lane shuffles); quarter h of the wave
//           forms A rows [8 h, 8 h + 8) and B columns [4 h, 4 h + 4) from one
//           exact anchor each (phase reduced in FP64) and complex-multiply
//           steps (at most 7), splits them, and writes them into the
//           operand slots of the wave's LDS table;
//   sum     lanes run over operand slots: per 8-ray block four 16-byte LDS
//           reads and three MFMAs.
// The geometry of the next super-group is loaded before the groups run, so its
// global loads are in flight while the groups are summed.  The MFMA
// accumulates one super-group (64 rays); super-group sums are added into a
// second accumulator, which keeps the float32 sums short.  Waves combine through LDS in a fixed
// order.
__global__ __launch_bounds__(kThreads) void synth_kernel(SynthArgs a) {
    __shared__ uint4 lds_raw[kWaves * kTableWords / 4];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // XCD-aware order: consecutive workgroup ids are dealt round-robin to the
    // 8 XCDs, so give each XCD a contiguous run of (pair, pass, partition,
    // chirp) blocks.  The pairs of one partition and chirp, which read the
    // same ray geometry, then run side by side on one XCD and share its L2.
    int g = (gridDim.x & 7) ? (int)blockIdx.x
                            : (int)((blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3));
    const int q = g % a.n_pairs;
    g /= a.n_pairs;
    const int pass = g % a.n_passes;
    g /= a.n_passes;
    const int part = g % a.n_parts;
    const int jj = g / a.n_parts;
    const double* pq = a.pairs + 6 * q;
    uint32_t* tw = reinterpret_cast<uint32_t*>(lds_raw) + wave * kTableWords;

    constexpr int kSplit = kWave / kGroup;           // lanes per ray in the build phase
    constexpr int kRowsPer = kRows / kSplit;         // A rows per lane (8)
    constexpr int kColsPer = kCols / kSplit;         // B columns per lane (4)
    const int ri = lane & (kGroup - 1);              // build: ray of the group
    const int h = lane / kGroup;                     // build: quarter of the rows and columns
    const int ma = pass * kRows + h * kRowsPer;      // first A row of the lane (global row index)
    const int ka = h * kColsPer;                     // first B column of the lane
    // build: where ray ri's operand values go (block, lane half, word in the slot)
    const int bk = ri / kBlockRays;
    const int hh = (ri % kBlockRays) / 4;
    const int rr = ri % 4;
    uint32_t* ahi = tw + bk * kBlockWords + rr;
    uint32_t* alo = ahi + kArrayWords;
    uint32_t* bhi = ahi + 2 * kArrayWords;
    uint32_t* blo = ahi + 3 * kArrayWords;
    const int la = h * kRowsPer + 32 * hh;           // slot of row h * 8 (+ t)
    const int lb = h * kColsPer + 32 * hh;           // slot of column h * 4 (+ t) ...
    const int lb2 = lb + kCols;                      // ... and of column 16 + h * 4 (+ t)

    f32x16 tot = {};
    const int r0 = part * a.rays_per_part;
    const int r1 = min(a.n_rays, r0 + a.rays_per_part);
    Geo gn = load_geo(a, r0 + wave * kWave + lane, r1, jj);
    for (int sbase = r0 + wave * kWave; sbase < r1; sbase += kThreads) {
        const Phases own = ray_phases(a, gn, pq);
        gn = load_geo(a, sbase + kThreads + lane, r1, jj);      // next super-group, in flight meanwhile
        const float2 own_s16 = cis(frac1(kCols * own.theta));   // step between rows
        const float2 own_s1 = cis(own.theta);                   // step between columns
        f32x16 acc[kGroup / kBlockRays] = {};   // one chain per block: consecutive MFMAs are independent
        for (int gq = 0; gq < kSplit && sbase + gq * kGroup < r1; ++gq) {
            const int src = gq * kGroup + ri;
            const double phi = __shfl(own.phi, src);
            const double theta = __shfl(own.theta, src);
            const float w = __shfl(own.w, src);
            const float2 s16 = make_float2(__shfl(own_s16.x, src), __shfl(own_s16.y, src));
            const float2 s1 = make_float2(__shfl(own_s1.x, src), __shfl(own_s1.y, src));
            {                                        // A rows ma + t: p_t = p_0 s^t
                float2 p = cis(frac1(phi + (double)ma * frac1(kCols * theta)));
                p.x *= w;
                p.y *= w;
#pragma unroll
                for (int t = 0; t < kRowsPer; ++t) {     // A'[m][0] = Re, A'[m][1] = Im
                    uint32_t hi, lo;
                    split2(p.x, p.y, hi, lo);
                    ahi[slot_word(la + t)] = hi;
                    alo[slot_word(la + t)] = lo;
                    p = cmul(p, s16);
                }
            }
            {                                        // B columns ka + t: q_t = q_0 s1^t
                float2 qv = cis(frac1((double)ka * theta));
#pragma unroll
                for (int t = 0; t < kColsPer; ++t) {
                    uint32_t hi, lo;
                    split2(qv.x, qv.y, hi, lo);
                    qv = cmul(qv, s1);
                    // column k: (B'[0][k], B'[1][k]) = (Re, -Im); column 16 + k: (Im, Re)
                    bhi[slot_word(lb + t)] = hi ^ 0x80000000u;
                    blo[slot_word(lb + t)] = lo ^ 0x80000000u;
                    bhi[slot_word(lb2 + t)] = (hi >> 16) | (hi << 16);
                    blo[slot_word(lb2 + t)] = (lo >> 16) | (lo << 16);
                }
            }
            __builtin_amdgcn_wave_barrier();
            // Every slot is written in every group; rays at or past the
            // partition end have A' = 0.
            constexpr int kB = kGroup / kBlockRays;
            f16x8 a_hi[kB], a_lo[kB], b_hi[kB], b_lo[kB];
#pragma unroll
            for (int b = 0; b < kB; ++b) {
                const uint32_t* base = tw + b * kBlockWords + slot_word(lane);
                a_hi[b] = *reinterpret_cast<const f16x8*>(base);
                a_lo[b] = *reinterpret_cast<const f16x8*>(base + kArrayWords);
                b_hi[b] = *reinterpret_cast<const f16x8*>(base + 2 * kArrayWords);
                b_lo[b] = *reinterpret_cast<const f16x8*>(base + 3 * kArrayWords);
            }
#pragma unroll
            for (int b = 0; b < kB; ++b) acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a_hi[b], b_hi[b], acc[b], 0, 0, 0);
#pragma unroll
            for (int b = 0; b < kB; ++b) acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a_hi[b], b_lo[b], acc[b], 0, 0, 0);
#pragma unroll
            for (int b = 0; b < kB; ++b) acc[b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(a_lo[b], b_hi[b], acc[b], 0, 0, 0);
            __builtin_amdgcn_wave_barrier();
        }
#pragma unroll
        for (int b = 0; b < kGroup / kBlockRays; ++b) tot += acc[b];
    }

    // Result layout of the 32 x 32 MFMA: register r of lane l holds row
    // 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32.  Row m, column col is
    // sample 16 m + col % 16 of the pass, real part for col < 16, imaginary
    // otherwise.  The wave sums reuse the table memory.
    __syncthreads();
    float* red = reinterpret_cast<float*>(lds_raw);
    const int c = lane >> 5, col = lane & 31;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int m = 8 * (r >> 2) + 4 * c + (r & 3);
        const int n = kCols * m + (col & (kCols - 1));
        red[wave * 2 * kBlock + 2 * n + (col >> 4)] = tot[r];
    }
    __syncthreads();
    float2* out = a.partial + (((int64_t)part * a.n_pairs + q) * a.chirp_count + jj) * (int64_t)a.n_samples;
    const int n_end = min(a.n_samples - pass * kBlock, kBlock);
    for (int n = threadIdx.x; n < n_end; n += kThreads) {
        float re = 0.f, im = 0.f;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            re += red[w * 2 * kBlock + 2 * n];
            im += red[w * 2 * kBlock + 2 * n + 1];
        }
        out[pass * kBlock + n] = make_float2(re, im);
    }
}

// Workgroup (pair q, partition p, chirp j) of the spreading method.  The
// workgroup's grid of M complex cells sits in LDS as 64-bit fixed-point
// integers (real parts, then imaginary parts) with the scale 2^e chosen from
// the largest weight, 2^e max|w| in [2^29, 2^30): every contribution
// w e^{2 pi i phi'} psi is cut to an int32 multiple of 2^-e (toward zero, error
// below 2^-29 max|w|) and added with a 64-bit LDS integer atomic; a cell of a block
// receives at most n_rays contributions, so no sum exceeds 2^60.  Integer
// addition is exact and order-free, so all waves share the grid and the result
// does not depend on scheduling (LDS float atomics would not be, and on this
// chip they are several times slower than integer ones).
//
// Each wave takes the partition's rays 64 at a time, one ray per lane (the
// same super-group order and geometry prefetch as synth_kernel): the lane forms
// the ray's phases in FP64, its grid position x = M theta, the first cell
// l0 = ceil(x - kTaps / 2) under the kernel and the offset
// s = l0 - x + (kTaps - 1) / 2 in [-1/2, 1/2), evaluates the kTaps kernel
// values by Horner's rule and adds the contributions into cells l0 .. l0 +
// kTaps - 1 (modulo M).  At the end the grid is scaled back and written as
// the partition's float32 grid.
__global__ __launch_bounds__(kThreads) void spread_kernel(SynthArgs a) {
    extern __shared__ unsigned long long gq[];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int M = 1 << a.grid_log2;
    // XCD-aware order as in synth_kernel: the pairs of one partition and chirp
    // run side by side on one XCD.
    int g = (gridDim.x & 7) ? (int)blockIdx.x
                            : (int)((blockIdx.x & 7) * (gridDim.x >> 3) + (blockIdx.x >> 3));
    const int q = g % a.n_pairs;
    g /= a.n_pairs;
    const int part = g % a.n_parts;
    const int jj = g / a.n_parts;
    const double* pq = a.pairs + 6 * q;
    // Each plane has kTaps cells of padding: padded cell i holds grid cell
    // (i - kTaps / 2) mod M, so a ray's taps are one address plus constant
    // offsets; the wrapped cells are folded back when the grid is written.
    // Even and odd lanes add into separate copies of the grid (2P + 1 cells
    // apart, so equal cells of the two copies sit in different banks): rays
    // of one target share cells, and two copies halve the lanes of one
    // atomic instruction that can meet on the same address.
    const int P = M + kTaps;
    const int CS = 2 * P + 1;
    for (int i = threadIdx.x; i < kGridCopies * CS; i += kThreads) gq[i] = 0ull;
    int e2;
    frexpf(__uint_as_float(*a.wmax_bits), &e2);     // max|w| = m 2^e2, m in [1/2, 1)
    const int qexp = 30 - e2;                       // 2^qexp max|w| in [2^29, 2^30)
    __syncthreads();

    const int r0 = part * a.rays_per_part;
    const int r1 = min(a.n_rays, r0 + a.rays_per_part);
    const double fM = (double)M;
    Geo gn = load_geo(a, r0 + wave * kWave + lane, r1, jj);
    for (int sbase = r0 + wave * kWave; sbase < r1; sbase += kThreads) {
        const Phases own = ray_phases(a, gn, pq);
        gn = load_geo(a, sbase + kThreads + lane, r1, jj);      // next super-group, in flight meanwhile
        if (own.w != 0.0f) {
            const double x = own.theta * fM;                   // grid position in [0, M)
            const double l0 = ceil(x - 0.5 * kTaps);
            const float sv = (float)((l0 - x) + 0.5 * (kTaps - 1));
            float2 c = cis(frac1(own.phi + frac1((double)a.center * own.theta)));
            const float ws = ldexpf(own.w, qexp);             // weight in grid units (exact)
            c.x *= ws;
            c.y *= ws;
            // Kernel values, the mirrored taps t and kTaps - 1 - t from one
            // Horner pass over the even and odd parts in s^2.
            const float y = sv * sv;
            float k[kTaps];
#pragma unroll
            for (int t = 0; t < kTaps / 2; ++t) {
                float ev = a.tap_even[t][kTapDeg / 2];
#pragma unroll
                for (int d = kTapDeg / 2 - 1; d >= 0; --d) ev = fmaf(ev, y, a.tap_even[t][d]);
                float od = a.tap_odd[t][kTapDeg / 2 - 1];
#pragma unroll
                for (int d = kTapDeg / 2 - 2; d >= 0; --d) od = fmaf(od, y, a.tap_odd[t][d]);
                k[t] = fmaf(sv, od, ev);
                k[kTaps - 1 - t] = fmaf(-sv, od, ev);
            }
            // l0 is in [-kTaps / 2, M - kTaps / 2] for every finite theta in
            // [0, 1) (the clamp only guards non-finite pair coordinates), so
            // the taps' padded cells l0 + kTaps / 2 + t lie in [0, M + kTaps).
            const int base = min(max((int)l0, -kTaps / 2), M - kTaps / 2);
            unsigned long long* cr = gq + (lane & (kGridCopies - 1)) * CS + (base + kTaps / 2);
            unsigned long long* ci = cr + P;
#pragma unroll
            for (int t = 0; t < kTaps; ++t) {
                // |k c| < 2^31 by the choice of qexp; conversion rounds toward zero
                const long long vr = (int)(k[t] * c.x);
                const long long vi = (int)(k[t] * c.y);
                atomicAdd(cr + t, (unsigned long long)vr);
                atomicAdd(ci + t, (unsigned long long)vi);
            }
        }
    }
    __syncthreads();
    float2* out = a.partial + (((int64_t)part * a.n_pairs + q) * a.chirp_count + jj) * (int64_t)M;
    for (int i = threadIdx.x; i < M; i += kThreads) {
        const int h = i + kTaps / 2;                        // padded cell of grid cell i
        long long re = 0, im = 0;
#pragma unroll
        for (int cp = 0; cp < kGridCopies; ++cp) {
            const unsigned long long* g0 = gq + cp * CS;
            re += (long long)g0[h];
            im += (long long)g0[P + h];
            if (i < kTaps / 2) {                            // wrapped past the end
                re += (long long)g0[h + M];
                im += (long long)g0[P + h + M];
            }
            if (i >= M - kTaps / 2) {                       // wrapped below the start
                re += (long long)g0[h - M];
                im += (long long)g0[P + h - M];
            }
        }
        out[i] = make_float2((float)ldexp((double)re, -qexp), (float)ldexp((double)im, -qexp));
    }
}

// *bits = the float bits of max_i |w_i| (nonnegative floats order like their
// bit patterns); *bits must be zero on entry.  256 threads per block; one
// atomic per block.
__global__ __launch_bounds__(256) void wmax_kernel(const float* __restrict__ w, int n, unsigned* bits) {
    __shared__ unsigned wave_max[256 / kWave];
    unsigned m = 0u;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        m = max(m, __float_as_uint(fabsf(w[i])));
    for (int off = kWave / 2; off > 0; off >>= 1) m = max(m, (unsigned)__shfl_xor((int)m, off));
    if ((threadIdx.x & (kWave - 1)) == 0) wave_max[threadIdx.x / kWave] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < 256 / kWave; ++k) m = max(m, wave_max[k]);
        atomicMax(bits, m);
    }
}

__global__ void set_u32_kernel(unsigned* p, unsigned v) { *p = v; }

// deconv[n] = 1 / psi_hat((n - center) / M), psi_hat(xi) the integral of
// psi(u) cos(2 pi xi u) over the kernel's support |u| <= kTaps / 2 (psi is
// even), by the trapezoid rule with kQuad intervals in FP64 (psi falls to
// e^{-beta} at the ends of its support, where the rule's error vanishes with
// it).  One wave per n; the lanes' partial sums are combined in a fixed order.
__global__ __launch_bounds__(kWave) void deconv_kernel(double* deconv, int n_samples, int center, int grid_log2) {
    const int n = blockIdx.x;
    const int lane = threadIdx.x;
    const double xi = (double)(n - center) / (double)(1 << grid_log2);
    const double h = (double)kTaps / kQuad;
    double acc = 0.0;
    for (int i = lane; i <= kQuad; i += kWave) {
        const double u = -0.5 * kTaps + i * h;
        const double z = 2.0 * u / kTaps;
        const double psi = exp(kBeta * (sqrt(fmax(0.0, 1.0 - z * z)) - 1.0));
        acc += ((i == 0 || i == kQuad) ? 0.5 * h : h) * psi * cospi(2.0 * xi * u);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    if (lane == 0 && n < n_samples) deconv[n] = 1.0 / acc;
}

// Workgroup (pair q, batch chirp j): the partitions' grids of the block summed
// in FP64 in partition order, loaded bit-reversed; the inverse DFT
// G[m] = sum_l g[l] e^{2 pi i m l / M} by radix-2 decimation in time in FP64
// in LDS (twiddles from sincospi); then s[n] = G[(n - center) mod M] deconv[n]
// rounded once to float32 and written into the cube at chirp c0 + j.
constexpr int kFinishThreads = 1024;     // one grid cell per thread at M = 1024

__global__ __launch_bounds__(kFinishThreads) void finish_kernel(SynthArgs a, float2* __restrict__ s, int n_chirps_out,
                                                              int c0) {
    extern __shared__ double2 fl[];
    const int logL = a.grid_log2, L = 1 << logL;
    double2* tw = fl;                    // L / 2 twiddles e^{+2 pi i k / L}
    double2* x = fl + L / 2;
    const int q = blockIdx.x % a.n_pairs, jj = blockIdx.x / a.n_pairs;
    for (int k = threadIdx.x; k < L / 2; k += blockDim.x) {
        double sn, cs;
        sincospi(2.0 * k / L, &sn, &cs);
        tw[k] = make_double2(cs, sn);
    }
    const int64_t stride = (int64_t)a.n_pairs * a.chirp_count * L;
    const float2* src = a.partial + ((int64_t)q * a.chirp_count + jj) * L;
    for (int l = threadIdx.x; l < L; l += blockDim.x) {
        double re = 0.0, im = 0.0;
#pragma unroll 4
        for (int p = 0; p < a.n_parts; ++p) {
            const float2 v = src[(int64_t)p * stride + l];
            re += v.x;
            im += v.y;
        }
        x[__brev((unsigned)l) >> (32 - logL)] = make_double2(re, im);
    }
    __syncthreads();
    for (int st = 0; st < logL; ++st) {
        const int half = 1 << st;
        for (int k = threadIdx.x; k < L / 2; k += blockDim.x) {
            const int pos = k & (half - 1);
            const int i0 = ((k >> st) << (st + 1)) + pos, i1 = i0 + half;
            const double2 w = tw[pos << (logL - 1 - st)];
            const double2 u = x[i0], v = x[i1];
            const double vr = v.x * w.x - v.y * w.y, vi = v.x * w.y + v.y * w.x;
            x[i0] = make_double2(u.x + vr, u.y + vi);
            x[i1] = make_double2(u.x - vr, u.y - vi);
        }
        __syncthreads();
    }
    float2* out = s + ((int64_t)q * n_chirps_out + c0 + jj) * a.n_samples;
    for (int n = threadIdx.x; n < a.n_samples; n += blockDim.x) {
        const double2 v = x[(n - a.center) & (L - 1)];
        const double f = a.deconv[n];
        out[n] = make_float2((float)(v.x * f), (float)(v.y * f));
    }
}

__global__ void reduce_kernel(const float2* __restrict__ partial, float2* __restrict__ s, int n_pairs, int nb,
                              int n_samples, int n_parts, int n_chirps_out, int c0) {
    const int64_t count = (int64_t)n_pairs * nb * n_samples;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double re = 0.0, im = 0.0;
    for (int p = 0; p < n_parts; ++p) {
        const float2 v = partial[(int64_t)p * count + i];
        re += v.x;
        im += v.y;
    }
    const int n = (int)(i % n_samples);
    const int64_t qj = i / n_samples;
    const int jj = (int)(qj % nb), q = (int)(qj / nb);
    s[((int64_t)q * n_chirps_out + c0 + jj) * n_samples + n] = make_float2((float)re, (float)im);
}

// Radix-2 decimation-in-time FFT of `lines` lines of length L = 2^logL, M
// lines per workgroup held in LDS.  Line m starts at
//   (m / per_group) * group_stride + (m % per_group) * line_stride
// and its elements are elem_stride apart.  Twiddles exp(-2 pi i k / L) are
// formed in FP64 and rounded once.
__global__ __launch_bounds__(256) void fft_kernel(const float2* in, float2* out, int logL, int lines, int M,
                                                  int per_group, int64_t group_stride, int64_t line_stride,
                                                  int64_t elem_stride) {
    extern __shared__ float2 lds[];
    const int L = 1 << logL;
    float2* tw = lds;              // L / 2 twiddles
    float2* x = lds + L / 2;       // M lines
    for (int k = threadIdx.x; k < L / 2; k += blockDim.x) {
        double sn, cs;
        sincospi(-2.0 * k / L, &sn, &cs);
        tw[k] = make_float2((float)cs, (float)sn);
    }
    const int m0 = blockIdx.x * M;
    const int nm = min(M, lines - m0);
    // load, bit-reversed within each line.  Consecutive threads take
    // consecutive elements of a contiguous line, or the same element of
    // neighbouring lines when the elements are strided.
    const bool by_elem = elem_stride == 1;
    for (int t = threadIdx.x; t < nm * L; t += blockDim.x) {
        const int ml = by_elem ? t / L : t % nm, e = by_elem ? t % L : t / nm;
        const int m = m0 + ml;
        const int64_t base = (int64_t)(m / per_group) * group_stride + (int64_t)(m % per_group) * line_stride;
        const int rev = logL ? (int)(__brev((unsigned)e) >> (32 - logL)) : 0;
        x[ml * L + rev] = in[base + (int64_t)e * elem_stride];
    }
    __syncthreads();
    for (int s = 0; s < logL; ++s) {
        const int half = 1 << s;
        for (int t = threadIdx.x; t < nm * (L / 2); t += blockDim.x) {
            const int ml = t / (L / 2), k = t % (L / 2);
            const int pos = k & (half - 1);
            const int i0 = ((k >> s) << (s + 1)) + pos;
            const int i1 = i0 + half;
            const float2 w = tw[pos << (logL - 1 - s)];
            float2* xl = x + ml * L;
            const float2 u = xl[i0], v = xl[i1];
            const float vr = v.x * w.x - v.y * w.y;
            const float vi = v.x * w.y + v.y * w.x;
            xl[i0] = make_float2(u.x + vr, u.y + vi);
            xl[i1] = make_float2(u.x - vr, u.y - vi);
        }
        __syncthreads();
    }
    for (int t = threadIdx.x; t < nm * L; t += blockDim.x) {
        const int ml = by_elem ? t / L : t % nm, e = by_elem ? t % L : t / nm;
        const int m = m0 + ml;
        const int64_t base = (int64_t)(m / per_group) * group_stride + (int64_t)(m % per_group) * line_stride;
        out[base + (int64_t)e * elem_stride] = x[ml * L + e];
    }
}

__global__ void span_kernel(rmd_scene sc, const uint8_t* __restrict__ in_set, rmd_span_rule rule,
                            const float* __restrict__ amp, float* __restrict__ weights) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= sc.n_rays) return;
    const int32_t b = sc.ray_off[i], e = sc.ray_off[i + 1];
    bool ok = b >= 0 && e <= sc.n_hits && e >= b;
    int inside = 0, n = 0;
    if (ok) {
        for (int64_t k = b; k < e; ++k) {
            const int32_t m = sc.hit_mesh[k];
            if (m < 0 || m >= sc.n_meshes) { ok = false; break; }
            inside += in_set[m] != 0;
            ++n;
        }
    }
    if (ok) {
        if (rule.mode == 0) ok = inside > 0;
        else if (rule.mode == 1) ok = inside == 0;
        else ok = inside == n;
        ok = ok && n >= rule.min_hits && n <= rule.max_hits;
    }
    weights[i] = ok ? (amp ? amp[i] : 1.0f) : 0.0f;
}

__global__ void zero_kernel(unsigned long long* p) { *p = 0ull; }

__global__ void check_kernel(SynthArgs a, unsigned long long* bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n_rays) return;
    const int32_t b = a.ray_off[i], e = a.ray_off[i + 1];
    bool ok = b >= 0 && e <= a.n_hits && e >= b;
    for (int64_t k = b; ok && k < e; ++k) {
        double x, y, z;
        ok = hit_point(a, a.verts, k, x, y, z);
    }
    if (!ok) atomicAdd(bad, 1ull);
}

}  // namespace rmd

// ------------------------------------------------------------------ C ABI

namespace {

thread_local std::string g_err;

rmd_status fail(rmd_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

rmd_status hip_fail(hipError_t e, const char* what) {
    return fail(RMD_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

rmd_status check_scene_desc(const rmd_scene* sc) {
    if (!sc) return fail(RMD_EINVAL, "scene is NULL");
    if (sc->n_meshes <= 0 || sc->n_tris <= 0 || sc->n_verts <= 0 || sc->n_rays <= 0 || sc->n_hits < 0)
        return fail(RMD_EINVAL, "scene sizes must be positive (n_hits >= 0)");
    if (sc->n_hits > INT32_MAX) return fail(RMD_EINVAL, "n_hits above 2^31 - 1 (32-bit ray offsets)");
    if (sc->n_rays > RMD_MAX_RAYS) return fail(RMD_EINVAL, "n_rays above RMD_MAX_RAYS");
    if (!sc->mesh_tri_off || !sc->tris || !sc->verts || !sc->ray_off || !sc->hit_mesh || !sc->hit_tri ||
        !sc->hit_u || !sc->hit_v)
        return fail(RMD_EINVAL, "a scene array pointer is NULL");
    return RMD_OK;
}

// Work plan of one IF cube.  Chirps are processed in batches whose per-ray
// geometry (7 doubles per ray and chirp) fits in kGeoBudget bytes, at most
// kMaxBatch chirps.  Within a batch the rays are split into partitions so that
// the (pair, chirp, partition) workgroups fill the device several times over,
// each wave keeping at least four 64-ray super-groups.  The workspace holds the
// batch's geometry, then the partition results of either method (direct:
// n_samples complex values per block; spreading: an M-cell grid per block and
// the deconvolution table), so one size serves both entry points.
constexpr int64_t kGeoBudget = int64_t(1) << 30;
constexpr int kMaxBatch = 16;

int grid_log2_for(int n_samples) {
    int l = rmd::kMinGridLog2;
    while ((1 << l) < 2 * n_samples) ++l;
    return l;
}

int64_t round256(int64_t b) { return (b + 255) / 256 * 256; }

struct Plan {
    int batch, parts, rays_per_part, grid_log2;
    int64_t geo_bytes, rec_bytes, partial_bytes, grid_bytes, deconv_bytes, total_bytes;
    int geo_sets;   // geometry buffers: 2 when there are several batches (the next one is built meanwhile)
};

Plan plan(int n_rays, int64_t n_hits, int n_pairs, int chirp_count, int n_samples) {
    Plan p{};
    const int64_t per_chirp = (int64_t)n_rays * 7 * (int64_t)sizeof(double);
    p.batch = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)chirp_count, kMaxBatch, kGeoBudget / per_chirp}));
    const int64_t blocks = (int64_t)n_pairs * p.batch;
    const int64_t target = 8192;
    int64_t np = (target + blocks - 1) / blocks;
    const int64_t max_p = std::max<int64_t>(1, n_rays / (rmd::kThreads * 4));
    np = std::max<int64_t>(1, std::min(np, max_p));
    int64_t rpp = (n_rays + np - 1) / np;
    rpp = (rpp + rmd::kThreads - 1) / rmd::kThreads * rmd::kThreads;
    p.parts = (int)((n_rays + rpp - 1) / rpp);
    p.rays_per_part = (int)rpp;
    p.grid_log2 = grid_log2_for(n_samples);
    p.geo_bytes = round256(per_chirp * p.batch);
    p.rec_bytes = round256(n_hits * (int64_t)sizeof(int4)) + round256(n_hits * (int64_t)sizeof(float));
    p.partial_bytes = (int64_t)p.parts * blocks * n_samples * (int64_t)sizeof(float2);
    p.grid_bytes = round256((int64_t)p.parts * blocks * (int64_t(1) << p.grid_log2) * (int64_t)sizeof(float2));
    p.deconv_bytes = round256((int64_t)n_samples * (int64_t)sizeof(double)) + 256;   // + the max-weight word
    p.geo_sets = chirp_count > p.batch ? 2 : 1;
    p.total_bytes = p.geo_sets * p.geo_bytes + p.rec_bytes + std::max(p.partial_bytes, p.grid_bytes + p.deconv_bytes);
    return p;
}

// Monomial coefficients (in s in [-1/2, 1/2]) of the degree-kTapDeg
// polynomials that interpolate the spreading kernel of taps t < kTaps / 2 at
// the kTapDeg + 1 Chebyshev points of that interval (tap t sits u = s + 1/2 -
// kTaps/2 + t cells from the ray; the nodes are symmetric, so the mirrored tap
// kTaps - 1 - t is the same polynomial at -s), split into even and odd parts.
// Solved once, in long double, by Gaussian elimination with partial pivoting.
struct TapPoly {
    float even[rmd::kTaps / 2][rmd::kTapDeg / 2 + 1];
    float odd[rmd::kTaps / 2][rmd::kTapDeg / 2];
};

const TapPoly& tap_poly() {
    static const TapPoly tp = [] {
        TapPoly r{};
        constexpr int n = rmd::kTapDeg + 1;
        const long double pi = 3.141592653589793238462643383279502884L;
        for (int t = 0; t < rmd::kTaps / 2; ++t) {
            long double A[n][n + 1];
            for (int i = 0; i < n; ++i) {
                const long double sn = 0.5L * cosl(pi * (i + 0.5L) / n);
                const long double z = (sn + 0.5L - 0.5L * rmd::kTaps + t) * 2.0L / rmd::kTaps;
                long double pw = 1.0L;
                for (int j = 0; j < n; ++j) {
                    A[i][j] = pw;
                    pw *= sn;
                }
                A[i][n] = expl((long double)rmd::kBeta * (sqrtl(fmaxl(0.0L, 1.0L - z * z)) - 1.0L));
            }
            for (int col = 0; col < n; ++col) {
                int piv = col;
                for (int i = col + 1; i < n; ++i)
                    if (fabsl(A[i][col]) > fabsl(A[piv][col])) piv = i;
                for (int j = 0; j <= n; ++j) std::swap(A[col][j], A[piv][j]);
                for (int i = col + 1; i < n; ++i) {
                    const long double f = A[i][col] / A[col][col];
                    for (int j = col; j <= n; ++j) A[i][j] -= f * A[col][j];
                }
            }
            for (int i = n - 1; i >= 0; --i) {      // back substitution; x_j kept in A[j][n]
                long double v = A[i][n];
                for (int j = i + 1; j < n; ++j) v -= A[i][j] * A[j][n];
                A[i][n] = v / A[i][i];
            }
            for (int j = 0; j < n; ++j) {
                if (j % 2 == 0)
                    r.even[t][j / 2] = (float)A[j][n];
                else
                    r.odd[t][j / 2] = (float)A[j][n];
            }
        }
        return r;
    }();
    return tp;
}

// Workspace of rmd_if_cube_static: a file-scope device array (each GPU the
// library runs on holds its own copy for the life of the process).  Host code
// must not pass the array's name to a kernel or a copy (on the host it is a
// stand-in, not a device address): static_scratch() looks up the device
// address of the current device's copy once and keeps it.
static __device__ __align__(256) unsigned char scratch[RMD_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

rmd_status static_scratch(void** out) {
    static std::mutex mu;
    static void* addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(RMD_EINVAL, "device index beyond the static scratch table");
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(RMD_EHIP, "hipGetSymbolAddress(scratch) gave NULL");
        addr[dev] = p;
    }
    *out = addr[dev];
    return RMD_OK;
}

rmd::SynthArgs synth_args(const rmd_scene* sc) {
    rmd::SynthArgs a{};
    a.mesh_tri_off = sc->mesh_tri_off;
    a.tris = sc->tris;
    a.verts = sc->verts;
    a.ray_off = sc->ray_off;
    a.hit_mesh = sc->hit_mesh;
    a.hit_tri = sc->hit_tri;
    a.hit_u = sc->hit_u;
    a.hit_v = sc->hit_v;
    a.n_hits = sc->n_hits;
    a.n_meshes = sc->n_meshes;
    a.n_tris = sc->n_tris;
    a.n_verts = sc->n_verts;
    a.n_rays = sc->n_rays;
    return a;
}

}  // namespace

extern "C" {

int32_t rmd_api_version(void) { return 2; }

const char* rmd_last_error(void) { return g_err.c_str(); }

rmd_status rmd_check_scene(const rmd_scene* scene, int32_t n_chirps, void* workspace, int64_t* n_bad_rays,
                           hipStream_t stream) {
    rmd_status st = check_scene_desc(scene);
    if (st != RMD_OK) return st;
    if (n_chirps <= 0) return fail(RMD_EINVAL, "n_chirps must be positive");
    if (!workspace || !n_bad_rays) return fail(RMD_EINVAL, "workspace and n_bad_rays must not be NULL");
    (void)n_chirps;   // indices are checked against the first snapshot's layout (the same for all)
    rmd::SynthArgs a = synth_args(scene);
    auto* bad = static_cast<unsigned long long*>(workspace);
    hipLaunchKernelGGL(rmd::zero_kernel, dim3(1), dim3(1), 0, stream, bad);
    hipLaunchKernelGGL(rmd::check_kernel, dim3((scene->n_rays + 255) / 256), dim3(256), 0, stream, a, bad);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "check_kernel launch");
    unsigned long long h = 0;
    e = hipMemcpyAsync(&h, bad, sizeof(h), hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return hip_fail(e, "rmd_check_scene");
    *n_bad_rays = (int64_t)h;
    if (h) return fail(RMD_ESCENE, std::to_string(h) + " ray(s) with out-of-range meta data");
    return RMD_OK;
}

rmd_status rmd_workspace_bytes(const rmd_scene* scene, const rmd_radar* radar, int32_t n_pairs,
                               int32_t chirp_count, int64_t* bytes) {
    rmd_status st = check_scene_desc(scene);
    if (st != RMD_OK) return st;
    if (!radar || !bytes) return fail(RMD_EINVAL, "radar and bytes must not be NULL");
    if (n_pairs <= 0 || chirp_count <= 0 || radar->n_samples <= 0 || radar->n_samples > RMD_MAX_SAMPLES)
        return fail(RMD_EINVAL, "n_pairs, chirp_count must be positive; n_samples in [1, RMD_MAX_SAMPLES]");
    *bytes = plan(scene->n_rays, scene->n_hits, n_pairs, chirp_count, radar->n_samples).total_bytes;
    return RMD_OK;
}

}  // extern "C"

namespace {

// Checks shared by both IF entry points; fills the plan and the kernel
// arguments common to both methods.
rmd_status cube_setup(const rmd_scene* scene, const rmd_radar* radar, int32_t n_pairs, const double* pairs,
                      const float* weights, int32_t chirp0, int32_t chirp_count, float* s, void* workspace,
                      int64_t workspace_bytes, Plan& p, rmd::SynthArgs& a) {
    int64_t need = 0;
    rmd_status st = rmd_workspace_bytes(scene, radar, n_pairs, chirp_count, &need);
    if (st != RMD_OK) return st;
    if (!pairs || !s || !workspace) return fail(RMD_EINVAL, "pairs, s and workspace must not be NULL");
    if (workspace_bytes < need) return fail(RMD_EINVAL, "workspace smaller than rmd_workspace_bytes");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(RMD_EINVAL, "workspace not 256-byte aligned");
    if (radar->n_chirps <= 0 || chirp0 < 0 || chirp0 + (int64_t)chirp_count > radar->n_chirps)
        return fail(RMD_EINVAL, "chirp range outside [0, n_chirps)");
    if (!(radar->f_s > 0) || !(radar->t_chirp > 0) || !std::isfinite(radar->f_c) || !std::isfinite(radar->bandwidth))
        return fail(RMD_EINVAL, "radar parameters must be finite, f_s and t_chirp positive");
    p = plan(scene->n_rays, scene->n_hits, n_pairs, chirp_count, radar->n_samples);
    if ((int64_t)n_pairs * p.batch * p.parts * 2 > INT32_MAX) return fail(RMD_EINVAL, "too many (pair, chirp) blocks");

    a = synth_args(scene);
    a.pairs = pairs;
    a.weights = weights;
    a.geo = static_cast<double*>(workspace);
    const int64_t geo_all = p.geo_sets * p.geo_bytes;
    a.hit_rec = reinterpret_cast<int4*>(static_cast<char*>(workspace) + geo_all);
    a.hit_rec_v = reinterpret_cast<float*>(static_cast<char*>(workspace) + geo_all +
                                           round256(scene->n_hits * (int64_t)sizeof(int4)));
    a.partial = reinterpret_cast<float2*>(static_cast<char*>(workspace) + geo_all + p.rec_bytes);
    a.n_pairs = n_pairs;
    a.n_samples = radar->n_samples;
    a.n_parts = p.parts;
    a.rays_per_part = p.rays_per_part;
    a.n_passes = (radar->n_samples + rmd::kBlock - 1) / rmd::kBlock;
    const double mu = radar->bandwidth / radar->t_chirp;               // Eq. 3
    a.cyc_per_m = radar->f_c / rmd::kC0;
    a.step_per_m = mu / (rmd::kC0 * radar->f_s);
    return RMD_OK;
}

// Helper stream of the current device (created once, default priority): the
// geometry of the next chirp batch is built on it while the current batch is
// synthesised on the caller's stream.
rmd_status helper_stream(hipStream_t* out) {
    static std::mutex mu;
    static hipStream_t streams[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(RMD_EINVAL, "device index beyond the helper stream table");
    std::lock_guard<std::mutex> lock(mu);
    if (!streams[dev]) {
        e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
        if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
    }
    *out = streams[dev];
    return RMD_OK;
}

// The chirp batches of one IF cube: geometry_kernel of batch b into geometry
// set b mod geo_sets, then work(args, nb, c0) on `stream` (the batch's
// synthesis).  With two sets, batch b + 1's geometry runs on the helper stream
// while batch b is synthesised; events order each geometry after the
// synthesis that last read its set, and each synthesis after its geometry, so
// the helper stream's work is joined back into `stream` (also under graph
// capture).  The results are those of the serial order.
template <class Work>
rmd_status run_batches(const Plan& p, rmd::SynthArgs a, int32_t chirp0, int32_t chirp_count, int n_rays,
                       hipStream_t stream, Work&& work) {
    char* geo0 = reinterpret_cast<char*>(a.geo);
    auto geometry = [&](int b, hipStream_t st) {
        rmd::SynthArgs g = a;
        const int c0 = b * p.batch;
        g.chirp0 = chirp0 + c0;
        g.chirp_count = std::min(p.batch, chirp_count - c0);
        g.geo = reinterpret_cast<double*>(geo0 + (size_t)(b % p.geo_sets) * p.geo_bytes);
        hipLaunchKernelGGL(rmd::geometry_kernel, dim3((n_rays + 255) / 256, g.chirp_count), dim3(256), 0, st, g);
    };
    auto batch_args = [&](int b) {
        rmd::SynthArgs w = a;
        const int c0 = b * p.batch;
        w.chirp0 = chirp0 + c0;
        w.chirp_count = std::min(p.batch, chirp_count - c0);
        w.geo = reinterpret_cast<double*>(geo0 + (size_t)(b % p.geo_sets) * p.geo_bytes);
        return w;
    };
    const int nbatch = (chirp_count + p.batch - 1) / p.batch;
    if (p.geo_sets == 1) {
        for (int b = 0; b < nbatch; ++b) {
            geometry(b, stream);
            const rmd::SynthArgs w = batch_args(b);
            work(w, w.chirp_count, b * p.batch);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return hip_fail(e, "IF cube launch");
        }
        return RMD_OK;
    }
    hipStream_t s2 = nullptr;
    rmd_status st = helper_stream(&s2);
    if (st != RMD_OK) return st;
    hipEvent_t ev[5] = {};   // start, geometry done (per set), synthesis done (per set)
    for (auto& x : ev) {
        hipError_t e = hipEventCreateWithFlags(&x, hipEventDisableTiming);
        if (e != hipSuccess) {
            for (auto& y : ev)
                if (y) (void)hipEventDestroy(y);
            return hip_fail(e, "hipEventCreateWithFlags");
        }
    }
    hipEvent_t* geo_done = ev + 1;
    hipEvent_t* work_done = ev + 3;
    hipError_t e = hipEventRecord(ev[0], stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s2, ev[0], 0);      // after everything queued before the call
    if (e == hipSuccess) {
        geometry(0, s2);
        e = hipEventRecord(geo_done[0], s2);
    }
    for (int b = 0; b < nbatch && e == hipSuccess; ++b) {
        e = hipStreamWaitEvent(stream, geo_done[b & 1], 0);
        if (e != hipSuccess) break;
        const rmd::SynthArgs w = batch_args(b);
        work(w, w.chirp_count, b * p.batch);
        e = hipEventRecord(work_done[b & 1], stream);
        if (e != hipSuccess || b + 1 >= nbatch) break;
        // set (b + 1) % 2 was last read by batch b - 1
        if (b >= 1) e = hipStreamWaitEvent(s2, work_done[(b + 1) & 1], 0);
        if (e != hipSuccess) break;
        geometry(b + 1, s2);
        e = hipEventRecord(geo_done[(b + 1) & 1], s2);
    }
    if (e == hipSuccess) e = hipGetLastError();
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (e != hipSuccess) return hip_fail(e, "IF cube launch");
    return RMD_OK;
}

// Resolves the hits into a.hit_rec once per call (both methods).
rmd_status resolve_hits(const rmd::SynthArgs& a, hipStream_t stream) {
    if (a.n_hits > 0)
        hipLaunchKernelGGL(rmd::resolve_kernel, dim3((unsigned)((a.n_hits + 255) / 256)), dim3(256), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "resolve_kernel launch");
    return RMD_OK;
}

}  // namespace

extern "C" {

rmd_status rmd_if_cube(const rmd_scene* scene, const rmd_radar* radar, int32_t n_pairs, const double* pairs,
                       const float* weights, int32_t chirp0, int32_t chirp_count, float* s, void* workspace,
                       int64_t workspace_bytes, hipStream_t stream) {
    Plan p;
    rmd::SynthArgs a;
    rmd_status st = cube_setup(scene, radar, n_pairs, pairs, weights, chirp0, chirp_count, s, workspace,
                               workspace_bytes, p, a);
    if (st != RMD_OK) return st;
    st = resolve_hits(a, stream);
    if (st != RMD_OK) return st;
    const int M = 1 << p.grid_log2;
    a.grid_log2 = p.grid_log2;
    a.center = radar->n_samples / 2;
    char* tail = static_cast<char*>(workspace) + p.geo_sets * p.geo_bytes + p.rec_bytes + p.grid_bytes;
    auto* wmax = reinterpret_cast<unsigned*>(tail);
    auto* deconv = reinterpret_cast<double*>(tail + 256);
    a.deconv = deconv;
    a.wmax_bits = wmax;
    std::memcpy(a.tap_even, tap_poly().even, sizeof(a.tap_even));
    std::memcpy(a.tap_odd, tap_poly().odd, sizeof(a.tap_odd));
    hipLaunchKernelGGL(rmd::deconv_kernel, dim3(radar->n_samples), dim3(rmd::kWave), 0, stream, deconv,
                       radar->n_samples, a.center, a.grid_log2);
    if (weights) {
        hipLaunchKernelGGL(rmd::set_u32_kernel, dim3(1), dim3(1), 0, stream, wmax, 0u);
        const int blocks = (int)std::min<int64_t>(1024, (scene->n_rays + 255) / 256);
        hipLaunchKernelGGL(rmd::wmax_kernel, dim3(blocks), dim3(256), 0, stream, weights, scene->n_rays, wmax);
    } else {
        hipLaunchKernelGGL(rmd::set_u32_kernel, dim3(1), dim3(1), 0, stream, wmax, 0x3f800000u);   // 1.0f
    }
    const size_t spread_lds =
        (size_t)rmd::kGridCopies * (2 * (M + rmd::kTaps) + 1) * sizeof(unsigned long long);
    const size_t finish_lds = (size_t)(M / 2 + M) * sizeof(double2);
    // Chirp batches: the spreading and the transform of each batch after its
    // geometry (the partition count is the same for every batch: a shorter
    // last batch uses part of the buffers).
    return run_batches(p, a, chirp0, chirp_count, scene->n_rays, stream,
                       [&](const rmd::SynthArgs& w, int nb, int c0) {
                           const dim3 grid((unsigned)((int64_t)n_pairs * nb * p.parts));
                           hipLaunchKernelGGL(rmd::spread_kernel, grid, dim3(rmd::kThreads), spread_lds, stream, w);
                           hipLaunchKernelGGL(rmd::finish_kernel, dim3((unsigned)(n_pairs * nb)),
                                              dim3(rmd::kFinishThreads), finish_lds, stream, w,
                                              reinterpret_cast<float2*>(s), chirp_count, c0);
                       });
}

rmd_status rmd_if_cube_static(const rmd_scene* scene, const rmd_radar* radar, int32_t n_pairs, const double* pairs,
                              const float* weights, int32_t chirp0, int32_t chirp_count, float* s,
                              hipStream_t stream) {
    int64_t need = 0;
    rmd_status st = rmd_workspace_bytes(scene, radar, n_pairs, chirp_count, &need);
    if (st != RMD_OK) return st;
    if (need > RMD_STATIC_SCRATCH_BYTES)
        return fail(RMD_EINVAL, "rmd_if_cube_static: these sizes need " + std::to_string(need) +
                                    " bytes of workspace, the static scratch holds " +
                                    std::to_string((long long)RMD_STATIC_SCRATCH_BYTES));
    void* ws = nullptr;
    st = static_scratch(&ws);
    if (st != RMD_OK) return st;
    return rmd_if_cube(scene, radar, n_pairs, pairs, weights, chirp0, chirp_count, s, ws, RMD_STATIC_SCRATCH_BYTES,
                       stream);
}

rmd_status rmd_if_cube_direct(const rmd_scene* scene, const rmd_radar* radar, int32_t n_pairs, const double* pairs,
                              const float* weights, int32_t chirp0, int32_t chirp_count, float* s, void* workspace,
                              int64_t workspace_bytes, hipStream_t stream) {
    Plan p;
    rmd::SynthArgs a;
    rmd_status st = cube_setup(scene, radar, n_pairs, pairs, weights, chirp0, chirp_count, s, workspace,
                               workspace_bytes, p, a);
    if (st != RMD_OK) return st;
    st = resolve_hits(a, stream);
    if (st != RMD_OK) return st;
    // Chirp batches: the synthesis and the partition sums of each batch after
    // its geometry.
    const int n_samples = radar->n_samples;
    return run_batches(p, a, chirp0, chirp_count, scene->n_rays, stream,
                       [&](const rmd::SynthArgs& w, int nb, int c0) {
                           const dim3 grid((unsigned)((int64_t)n_pairs * w.n_passes * nb * p.parts));
                           hipLaunchKernelGGL(rmd::synth_kernel, grid, dim3(rmd::kThreads), 0, stream, w);
                           const int64_t count = (int64_t)n_pairs * nb * n_samples;
                           hipLaunchKernelGGL(rmd::reduce_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0,
                                              stream, w.partial, reinterpret_cast<float2*>(s), n_pairs, nb, n_samples,
                                              p.parts, chirp_count, c0);
                       });
}

rmd_status rmd_range_doppler(const float* s, float* S, int32_t n_pairs, int32_t n_chirps, int32_t n_samples,
                             hipStream_t stream) {
    if (!s || !S) return fail(RMD_EINVAL, "s and S must not be NULL");
    auto pow2 = [](int32_t n) { return n > 0 && (n & (n - 1)) == 0; };
    if (n_pairs <= 0 || !pow2(n_chirps) || !pow2(n_samples) || n_chirps > RMD_MAX_FFT || n_samples > RMD_MAX_FFT)
        return fail(RMD_EINVAL, "n_pairs > 0; n_chirps and n_samples powers of two <= RMD_MAX_FFT");
    if ((int64_t)n_pairs * n_chirps * n_samples > INT32_MAX) return fail(RMD_EINVAL, "cube too large");
    auto lg = [](int32_t n) { int l = 0; while ((1 << l) < n) ++l; return l; };
    const auto* in = reinterpret_cast<const float2*>(s);
    auto* out = reinterpret_cast<float2*>(S);
    // fast time: lines of n_samples, contiguous
    {
        const int L = n_samples, lines = n_pairs * n_chirps;
        const int M = std::max(1, std::min(lines, 2048 / L));
        const size_t lds = (size_t)(L / 2 + M * L) * sizeof(float2);
        hipLaunchKernelGGL(rmd::fft_kernel, dim3((lines + M - 1) / M), dim3(256), lds, stream, in, out, lg(L),
                           lines, M, 1, (int64_t)L, (int64_t)0, (int64_t)1);
    }
    // slow time: lines of n_chirps, n_samples apart; M neighbouring lines per block
    {
        const int L = n_chirps, lines = n_pairs * n_samples;
        const int M = std::max(1, std::min(n_samples, 2048 / L));
        const size_t lds = (size_t)(L / 2 + M * L) * sizeof(float2);
        hipLaunchKernelGGL(rmd::fft_kernel, dim3((lines + M - 1) / M), dim3(256), lds, stream, out, out, lg(L),
                           lines, M, n_samples, (int64_t)n_chirps * n_samples, (int64_t)1, (int64_t)n_samples);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "fft_kernel launch");
    return RMD_OK;
}

rmd_status rmd_span_weights(const rmd_scene* scene, const uint8_t* in_set, const rmd_span_rule* rule,
                            const float* amp, float* weights, hipStream_t stream) {
    rmd_status st = check_scene_desc(scene);
    if (st != RMD_OK) return st;
    if (!in_set || !rule || !weights) return fail(RMD_EINVAL, "in_set, rule and weights must not be NULL");
    if (rule->mode < 0 || rule->mode > 2) return fail(RMD_EINVAL, "span mode must be 0, 1 or 2");
    hipLaunchKernelGGL(rmd::span_kernel, dim3((scene->n_rays + 255) / 256), dim3(256), 0, stream, *scene, in_set,
                       *rule, amp, weights);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "span_kernel launch");
    return RMD_OK;
}

}  // extern "C"
