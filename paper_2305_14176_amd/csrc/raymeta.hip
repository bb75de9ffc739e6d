// libraymeta: radar IF synthesis from ray meta data (Section II, Eqs. 1-7)
// for gfx950.  The C ABI is declared in include/raymeta.h.
//
// Kernels:
//   synth_kernel   Eqs. 6, 7, 1, 2 fused: per workgroup one antenna pair, one
//                  chirp and one partition of the rays; FP64 geometry per ray,
//                  then an FP32 phasor recurrence over fast time.
//   reduce_kernel  sums the partitions' partial cubes in FP64, fixed order.
//   fft_kernel     radix-2 FFT of lines held in LDS (Eq. 4, one axis a pass).
//   span_kernel    Eq. 5 rule masks, one thread per ray.
//   check_kernel   counts rays with out-of-range meta data.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>

#include "raymeta.h"

namespace rmd {

constexpr int kWave = 64;
constexpr int kWaves = 4;                 // waves per synthesis workgroup
constexpr int kThreads = kWave * kWaves;
constexpr int kRun = 8;                   // consecutive fast-time samples per lane
constexpr int kBlock = kWave * kRun;      // samples one wave covers per pass (512)
constexpr int kHiBits = 16;               // bits of the split per-lane phase step
constexpr double kC0 = 299792458.0;

// One ray's contribution for one (pair, chirp), as the synthesis loop reads it.
//   phi    f_c tau modulo 1 (cycles): phase at t = 0
//   th_hi  kRun * theta modulo 1, rounded down to kHiBits fraction bits, with
//   th_lo  the rest: theta = mu tau / f_s is the phase step per sample (cycles)
//   w      weight (0: the ray contributes nothing)
//   cz, sz cos and sin of 2 pi theta;  c2 = 2 cos(2 pi theta)
struct alignas(16) Rec {
    float phi, th_hi, th_lo, w;
    float cz, sz, c2, pad;
};

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
    float2* partial;            // [n_parts][n_pairs][chirp_count][n_samples]
    int64_t n_hits;
    int32_t n_meshes, n_tris, n_verts, n_rays;
    int32_t n_pairs, chirp0, chirp_count, n_samples;
    int32_t n_parts, rays_per_part;
    double cyc_per_m;           // f_c / c: carrier cycles per metre of path (Eq. 1 into Eq. 2)
    double step_per_m;          // mu / (c f_s): beat cycles per sample per metre (Eqs. 1-3)
};

__device__ inline double dist3(double ax, double ay, double az, double bx, double by, double bz) {
    const double dx = ax - bx, dy = ay - by, dz = az - bz;
    return sqrt(dx * dx + dy * dy + dz * dz);
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

// Path length of ray i for pair q on chirp j's snapshot: inner path over the
// hits plus the two displaced antenna legs.  Returns false when the ray has no
// usable path (no hits, or out-of-range meta data).
__device__ bool ray_length(const SynthArgs& a, int ray, int j, const double* __restrict__ pq, double& len) {
    const int32_t b = a.ray_off[ray], e = a.ray_off[ray + 1];
    if (b < 0 || e > a.n_hits || e <= b) return false;
    const double* v = a.verts + (int64_t)j * a.n_verts * 3;
    double fx, fy, fz, lx, ly, lz;
    if (!hit_point(a, v, b, fx, fy, fz)) return false;
    lx = fx; ly = fy; lz = fz;
    double inner = 0.0;
    for (int64_t k = b + 1; k < e; ++k) {
        double x, y, z;
        if (!hit_point(a, v, k, x, y, z)) return false;
        inner += dist3(x, y, z, lx, ly, lz);
        lx = x; ly = y; lz = z;
    }
    len = dist3(fx, fy, fz, pq[0], pq[1], pq[2]) + inner + dist3(lx, ly, lz, pq[3], pq[4], pq[5]);
    return true;
}

__device__ Rec make_record(const SynthArgs& a, int ray, int j, const double* __restrict__ pq) {
    Rec r;
    r.phi = r.th_hi = r.th_lo = r.w = r.sz = r.pad = 0.f;
    r.cz = 1.f;
    r.c2 = 2.f;
    double len;
    if (ray >= a.n_rays || !ray_length(a, ray, j, pq, len)) return r;
    const double wt = a.weights ? (double)a.weights[ray] : 1.0;
    const double ph = len * a.cyc_per_m;              // f_c tau, cycles
    double th = len * a.step_per_m;                   // mu tau / f_s, cycles per sample
    th -= floor(th);
    double thr = kRun * th;
    thr -= floor(thr);
    const double hi = floor(thr * (double)(1 << kHiBits)) * (1.0 / (double)(1 << kHiBits));
    double sn, cs;
    sincospi(2.0 * th, &sn, &cs);
    r.phi = (float)(ph - floor(ph));
    r.th_hi = (float)hi;                              // exact: kHiBits fraction bits
    r.th_lo = (float)(thr - hi);
    r.w = (float)wt;
    r.cz = (float)cs;
    r.sz = (float)sn;
    r.c2 = (float)(2.0 * cs);
    return r;
}

// Workgroup (pair q, chirp j, partition p): the rays of partition p are taken
// 64 at a time, one per lane, round-robin over the workgroup's waves.  Lane l
// of a wave first builds its ray's record (FP64 geometry) into the wave's LDS
// slice; the wave then walks the 64 records.  For each record, lane l owns the
// kRun consecutive samples n = 512 b + kRun l + r of each pass b: it evaluates
// the phasor at its first sample with the hardware sin/cos (argument in
// revolutions), its second by one complex multiply, and the rest with the
// two-term recurrence p_{r+1} = 2 cos(2 pi theta) p_r - p_{r-1}.  Sums of a
// 64-ray group are added into a second accumulator, which keeps the float32
// sums short.  Waves combine through LDS in a fixed order.
template <int NB>
__global__ __launch_bounds__(kThreads) void synth_kernel(SynthArgs a) {
    __shared__ Rec rec[kWaves][kWave];
    __shared__ float2 red[kWaves - 1][NB * kBlock];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    int g = blockIdx.x;
    const int q = g % a.n_pairs;
    g /= a.n_pairs;
    const int part = g % a.n_parts;
    const int jj = g / a.n_parts;
    const int j = a.chirp0 + jj;
    const double* pq = a.pairs + 6 * q;

    float2 tot[NB][kRun];
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int r = 0; r < kRun; ++r) tot[b][r] = make_float2(0.f, 0.f);

    float lf[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) lf[b] = (float)(b * kWave + lane);   // first sample / kRun

    const int r0 = part * a.rays_per_part;
    const int r1 = min(a.n_rays, r0 + a.rays_per_part);
    for (int base = r0 + wave * kWave; base < r1; base += kThreads) {
        rec[wave][lane] = make_record(a, base + lane, j, pq);
        __builtin_amdgcn_wave_barrier();
        float2 acc[NB][kRun];
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < kRun; ++r) acc[b][r] = make_float2(0.f, 0.f);
        const int cnt = min(kWave, r1 - base);
        for (int i = 0; i < cnt; ++i) {
            const Rec e = rec[wave][i];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                const float x = __builtin_amdgcn_fractf(lf[b] * e.th_hi);   // exact product
                const float ph = x + fmaf(lf[b], e.th_lo, e.phi);    // revolutions, [0, 2.01)
                float c0 = __builtin_amdgcn_cosf(ph);
                float s0 = __builtin_amdgcn_sinf(ph);
                float c1 = c0 * e.cz - s0 * e.sz;
                float s1 = c0 * e.sz + s0 * e.cz;
                acc[b][0].x = fmaf(e.w, c0, acc[b][0].x);
                acc[b][0].y = fmaf(e.w, s0, acc[b][0].y);
                acc[b][1].x = fmaf(e.w, c1, acc[b][1].x);
                acc[b][1].y = fmaf(e.w, s1, acc[b][1].y);
#pragma unroll
                for (int r = 2; r < kRun; ++r) {
                    const float c2 = fmaf(e.c2, c1, -c0);
                    const float s2 = fmaf(e.c2, s1, -s0);
                    acc[b][r].x = fmaf(e.w, c2, acc[b][r].x);
                    acc[b][r].y = fmaf(e.w, s2, acc[b][r].y);
                    c0 = c1; s0 = s1; c1 = c2; s1 = s2;
                }
            }
        }
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < kRun; ++r) {
                tot[b][r].x += acc[b][r].x;
                tot[b][r].y += acc[b][r].y;
            }
        __builtin_amdgcn_wave_barrier();
    }

    // Combine the waves: waves 1.. publish, wave 0 adds in wave order.
    if (wave > 0) {
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < kRun; ++r) red[wave - 1][b * kBlock + lane * kRun + r] = tot[b][r];
    }
    __syncthreads();
    if (wave == 0) {
        float2* out = a.partial +
                      (((int64_t)part * a.n_pairs + q) * a.chirp_count + jj) * (int64_t)a.n_samples;
#pragma unroll
        for (int b = 0; b < NB; ++b)
#pragma unroll
            for (int r = 0; r < kRun; ++r) {
                float2 v = tot[b][r];
                for (int w = 0; w < kWaves - 1; ++w) {
                    const float2 o = red[w][b * kBlock + lane * kRun + r];
                    v.x += o.x;
                    v.y += o.y;
                }
                const int n = b * kBlock + lane * kRun + r;
                if (n < a.n_samples) out[n] = v;
            }
    }
}

__global__ void reduce_kernel(const float2* __restrict__ partial, float2* __restrict__ s, int64_t count,
                              int n_parts) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    double re = 0.0, im = 0.0;
    for (int p = 0; p < n_parts; ++p) {
        const float2 v = partial[(int64_t)p * count + i];
        re += v.x;
        im += v.y;
    }
    s[i] = make_float2((float)re, (float)im);
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
    if (!sc->mesh_tri_off || !sc->tris || !sc->verts || !sc->ray_off || !sc->hit_mesh || !sc->hit_tri ||
        !sc->hit_u || !sc->hit_v)
        return fail(RMD_EINVAL, "a scene array pointer is NULL");
    return RMD_OK;
}

// Ray partitions: enough workgroups to fill the device several times over,
// each wave keeping at least four 64-ray groups.
void partition(int n_rays, int64_t pairs_chirps, int& n_parts, int& rays_per_part) {
    const int64_t target = 8192;
    int64_t p = (target + pairs_chirps - 1) / pairs_chirps;
    const int64_t max_p = std::max<int64_t>(1, n_rays / (rmd::kThreads * 4));
    p = std::max<int64_t>(1, std::min(p, max_p));
    int64_t rpp = (n_rays + p - 1) / p;
    rpp = (rpp + rmd::kThreads - 1) / rmd::kThreads * rmd::kThreads;
    n_parts = (int)((n_rays + rpp - 1) / rpp);
    rays_per_part = (int)rpp;
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

int32_t rmd_api_version(void) { return 1; }

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
    int parts, rpp;
    partition(scene->n_rays, (int64_t)n_pairs * chirp_count, parts, rpp);
    *bytes = (int64_t)parts * n_pairs * chirp_count * radar->n_samples * (int64_t)sizeof(float2);
    return RMD_OK;
}

rmd_status rmd_if_cube(const rmd_scene* scene, const rmd_radar* radar, int32_t n_pairs, const double* pairs,
                       const float* weights, int32_t chirp0, int32_t chirp_count, float* s, void* workspace,
                       int64_t workspace_bytes, hipStream_t stream) {
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
    const int64_t groups = (int64_t)n_pairs * chirp_count;
    int parts, rpp;
    partition(scene->n_rays, groups, parts, rpp);
    if (groups * parts > INT32_MAX) return fail(RMD_EINVAL, "too many (pair, chirp) blocks");

    rmd::SynthArgs a = synth_args(scene);
    a.pairs = pairs;
    a.weights = weights;
    a.partial = static_cast<float2*>(workspace);
    a.n_pairs = n_pairs;
    a.chirp0 = chirp0;
    a.chirp_count = chirp_count;
    a.n_samples = radar->n_samples;
    a.n_parts = parts;
    a.rays_per_part = rpp;
    const double mu = radar->bandwidth / radar->t_chirp;               // Eq. 3
    a.cyc_per_m = radar->f_c / rmd::kC0;
    a.step_per_m = mu / (rmd::kC0 * radar->f_s);
    const dim3 grid((unsigned)(groups * parts));
    if (radar->n_samples <= rmd::kBlock)
        hipLaunchKernelGGL(rmd::synth_kernel<1>, grid, dim3(rmd::kThreads), 0, stream, a);
    else
        hipLaunchKernelGGL(rmd::synth_kernel<2>, grid, dim3(rmd::kThreads), 0, stream, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "synth_kernel launch");
    const int64_t count = groups * radar->n_samples;
    hipLaunchKernelGGL(rmd::reduce_kernel, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, stream,
                       static_cast<const float2*>(workspace), reinterpret_cast<float2*>(s), count, parts);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "reduce_kernel launch");
    return RMD_OK;
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
