// Host side of the Yee FDTD library: context, validation, workspace carving,
// table construction and kernel launches behind the C ABI of include/yee.h.
//
// Definitions (the paper defines no full-wave solver; textbook operations):
//   dt  = S / (c0 sqrt(dx^-2 + dy^-2 + dz^-2))                  (Courant limit)
//   Ca  = (1 - s)/(1 + s), Cb = (dt/eps)/(1 + s), s = sigma dt/(2 eps)
//                                                  (Taflove & Hagness ch. 3)
//   CPML: x = depth/L, sigma = sigma_max x^m, kappa = 1 + (kappa_max - 1) x^m,
//         alpha = alpha_max (1 - x), b = exp(-(sigma/kappa + alpha) dt/eps0),
//         a = sigma (b - 1)/(kappa (sigma + kappa alpha))     (Roden & Gedney 2000);
//         the tables hold 1 - b, and psi <- b psi + a dF is evaluated as
//         psi - (1 - b) psi + a dF
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/yee.h"
#include "yee_adjoint.hpp"
#include "yee_kernels.hpp"
#include "yee_tb.hpp"

namespace {

constexpr double kC0 = 299792458.0;
constexpr double kPi = 3.14159265358979323846;
const double kMu0 = 4.0e-7 * kPi;
const double kEps0 = 1.0 / (kMu0 * kC0 * kC0);
const double kEta0 = std::sqrt(kMu0 / kEps0);

thread_local std::string g_err;

yee_status fail(yee_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t e_ = (expr);                                                        \
    if (e_ != hipSuccess)                                                          \
      return fail(YEE_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));        \
  } while (0)

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

#ifndef YEE_COMP_SKEW_BYTES
#define YEE_COMP_SKEW_BYTES 0
#endif

struct Region {
  size_t off = 0, bytes = 0;
};

}  // namespace

struct yee_ctx {
  yee_grid_desc d{};
  double dt = 0.0;
  int V = 1;        // x samples per lane
  int px = 0;       // x pitch in elements
  size_t tsize = 0; // storage element size
  size_t csize = 0; // compute element size
  int ty = 0, kz = 0, vpl = 0;  // launch shape (0 = automatic)
  int ty_req = 0, kz_req = 0;   // as requested by yee_set_launch
  // two steps per sweep: requested mode (0 automatic, 1 single steps only,
  // 2 required), its launch shape (0 = automatic) and whether it applies
  int tb_req = 0, tb_ty_req = 0, tb_kz_req = 0;
  int tb_ty = 0, tb_kz = 0, tb_V = 0, tb_wpr = 1;
  bool tb_ok = false;
  size_t lds_limit = 65536;  // per-workgroup LDS, queried at bind time

  // host-side configuration
  int nsx = 1, nsy = 1, nsz = 1;
  std::vector<int32_t> segx, segy, segz;
  std::vector<double> eps, sig;
  std::vector<int32_t> pec_k;
  std::vector<std::vector<uint8_t>> pec_masks;
  std::vector<yee::SrcDev> src;
  std::vector<int4> probes;
  std::vector<double> freqs;

  // workspace
  bool bound = false;
  unsigned char* ws = nullptr;
  int64_t ws_bytes = 0;
  Region fields[2], psi_e[2], psi_h[2], series, dft, stat, segr, coef, prof, pecplane, pecmask, rowflag,
      srcr, prober, freqr;
  size_t comp_bytes = 0;   // one component array
  size_t psi_len[6] = {};  // elements of each psi array (same for E and H side)
  uint32_t psi_off[6] = {};  // element offset of the pair array holding each psi auxiliary
  size_t prof_len = 0;     // elements of one profile array (max axis length)
  int64_t n = 0;           // steps taken
  int64_t folded = 0;      // steps folded into the DFT
  // current buffers: a single step and a two-step sweep both write the other
  // field set and H-side auxiliary set (cur); the E-side auxiliaries are
  // updated in place by a single step and ping-ponged by a sweep (pecur)
  int cur = 0, pecur = 0;
  bool in_batch = false;   // admitted to a batch (yee_load_state refuses)
  uint32_t* dbg_count = nullptr;   // debug write counts (single steps count their stores)
};

struct yee_batch {
  int32_t max_slots = 0;
  int32_t prec = YEE_F32;  // storage precision of every admitted context
  int64_t budget = 0;      // bytes of admitted context workspaces
  int32_t K = 0;           // steps per replay
  int32_t grid = 0;        // workgroups of the batched launch
  size_t lds = 0;
  unsigned char* ws = nullptr;
  int64_t ws_bytes = 0;
  bool bound = false;
  struct Slot {
    yee_ctx* ctx = nullptr;
    int64_t n_end = 0;     // step count at which the request is complete
    int64_t bytes = 0;
    int32_t ty = 0, kz = 0;
    bool used = false;
  };
  std::vector<Slot> slots;
  int64_t in_use = 0;
  // replay graphs, captured on first use: [0] cached stores, [1] stores
  // streamed past the last-level cache (active slots' fields exceed it)
  hipGraph_t graph[2] = {nullptr, nullptr};
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  hipStream_t capture = nullptr;       // private stream the replay graphs are captured on
  // host images of the descriptor table (pinned, used in turn; the event of
  // each marks the end of the copy that last read it)
  unsigned char* staging[2] = {nullptr, nullptr};
  hipEvent_t staged[2] = {nullptr, nullptr};
  bool staged_used[2] = {false, false};
  size_t staging_bytes = 0;
  int64_t runs = 0;
};

namespace {

constexpr int kMaxRow = 512;  // x samples per row a workgroup can cover

// Waves covering one row of nx samples at V samples per lane.
int waves_per_row(int nx, int V) { return (nx + yee::kWave * V - 1) / (yee::kWave * V); }

size_t storage_size(int prec) { return prec == YEE_F64 ? 8 : prec == YEE_F32 ? 4 : 2; }
size_t compute_size(int prec) { return prec == YEE_F64 ? 8 : 4; }

void psi_lengths(const yee_ctx* c, size_t out[6]) {
  const auto& d = c->d;
  const size_t px = c->px, ny = d.ny, nz = d.nz;
  const size_t lx = d.cpml_cells[0], ly = d.cpml_cells[1], lz = d.cpml_cells[2];
  // order: (comp, axis) = xy, xz, yz, yx, zx, zy  (same for E and H side)
  const size_t yl = nz * 2 * ly * px, zl = 2 * lz * ny * px, xl = nz * ny * 2 * lx;
  out[0] = yl; out[1] = zl; out[2] = zl; out[3] = xl; out[4] = xl; out[5] = yl;
}

void layout(yee_ctx* c) {
  const auto& d = c->d;
  size_t off = 0;
  auto take = [&](Region& r, size_t bytes) {
    r.off = off;
    r.bytes = bytes;
    off += align256(std::max<size_t>(bytes, 1));
  };
  // component arrays are skewed by an odd number of 256-byte units so that the
  // same (i, j, k) of the twelve streams does not land on one HBM channel
  // one zero plane after the last one: the march prefetches plane nz (the
  // tangential E above the top face, identically zero) without a branch
  c->comp_bytes = align256((size_t)(d.nz + 1) * d.ny * c->px * c->tsize) + YEE_COMP_SKEW_BYTES;
  for (int s = 0; s < 2; ++s) take(c->fields[s], 6 * c->comp_bytes);
  psi_lengths(c, c->psi_len);
  // the two auxiliaries of one axis are interleaved: pair arrays y (XY, ZY),
  // z (XZ, YZ), x (YX, ZX); psi_off[q] is the offset of q's pair array
  const size_t ypair = 2 * c->psi_len[0], zpair = 2 * c->psi_len[1], xpair = 2 * c->psi_len[3];
  c->psi_off[0] = c->psi_off[5] = 0;
  c->psi_off[1] = c->psi_off[2] = (uint32_t)ypair;
  c->psi_off[3] = c->psi_off[4] = (uint32_t)(ypair + zpair);
  const size_t psin = ypair + zpair + xpair;
  const size_t psib = psin * c->csize;
  take(c->psi_e[0], psib);
  take(c->psi_e[1], psib);
  take(c->psi_h[0], psib);
  take(c->psi_h[1], psib);
  const size_t np = c->probes.size(), nf = c->freqs.size();
  take(c->series, (size_t)d.series_len * np * sizeof(double));
  take(c->dft, np * nf * 2 * sizeof(double));
  take(c->stat, sizeof(uint32_t));   // status flags (yee_status_flags), last of the state run
  take(c->segr, ((size_t)c->px + d.ny + d.nz) * 4);
  take(c->coef, (size_t)c->nsx * c->nsy * c->nsz * 2 * c->csize);
  c->prof_len = std::max({d.nx, d.ny, d.nz}) + 1;
  take(c->prof, 2 * 3 * 3 * c->prof_len * c->csize);
  take(c->pecplane, (size_t)d.nz * 4);
  take(c->pecmask, c->pec_k.size() * (size_t)d.ny * c->px);
  take(c->rowflag, (size_t)d.nz * d.ny);
  take(c->srcr, c->src.size() * sizeof(yee::SrcDev));
  take(c->prober, np * sizeof(int4));
  take(c->freqr, nf * sizeof(double));
  c->ws_bytes = (int64_t)off;
}

// Roden-Gedney profile along one axis of n cells with a layer of L cells.
// side 0: E (positions 0..n-1 integer), side 1: H (positions i + 1/2).
// The decay factor is kept as omb = 1 - b (computed with expm1): near the
// inner edge of the layer b is within 1e-4 of 1, and in FP32 the difference
// would otherwise carry a relative error of order 1e-3.
void cpml_profile(const yee_grid_desc& d, double dw, double dt, int n, int L, int side,
                  std::vector<double>& omb, std::vector<double>& a, std::vector<double>& kinv) {
  omb.assign(n, 0.0);
  a.assign(n, 0.0);
  kinv.assign(n, 1.0);
  if (L <= 0) return;
  const double m = d.cpml_m;
  const double smax = d.cpml_sigma_max < 0.0 ? 0.8 * (m + 1.0) / (kEta0 * dw) : d.cpml_sigma_max;
  for (int i = 0; i < n; ++i) {
    const double p = i + (side ? 0.5 : 0.0);
    const double x = std::max(std::max((double)L - p, p - (double)(n - L)), 0.0) / L;
    const double xm = std::pow(x, m);
    const double sg = smax * xm;
    const double kp = 1.0 + (d.cpml_kappa_max - 1.0) * xm;
    const double al = d.cpml_alpha_max * (1.0 - x);
    const double om = -std::expm1(-(sg / kp + al) * dt / kEps0);
    const double den = kp * (sg + kp * al);
    omb[i] = om;
    a[i] = (sg > 0.0 && den > 0.0) ? -sg * om / den : 0.0;
    kinv[i] = 1.0 / kp;
  }
}

template <class C>
void put(std::vector<unsigned char>& buf, size_t byte_off, const std::vector<double>& v) {
  C* p = reinterpret_cast<C*>(buf.data() + byte_off);
  for (size_t i = 0; i < v.size(); ++i) p[i] = static_cast<C>(v[i]);
}

yee_status upload(yee_ctx* c, const Region& r, const void* host, size_t bytes, hipStream_t s) {
  if (bytes == 0) return YEE_OK;
  HIP_TRY(hipMemcpyAsync(c->ws + r.off, host, bytes, hipMemcpyHostToDevice, s));
  return YEE_OK;
}

yee_status upload_materials_impl(yee_ctx* c, hipStream_t s) {
  const size_t nb = (size_t)c->nsx * c->nsy * c->nsz;
  std::vector<double> cab(2 * nb);
  for (size_t b = 0; b < nb; ++b) {
    const double eps = kEps0 * c->eps[b];
    const double sg = c->sig[b] * c->dt / (2.0 * eps);
    cab[2 * b] = (1.0 - sg) / (1.0 + sg);
    cab[2 * b + 1] = (c->dt / eps) / (1.0 + sg);
  }
  std::vector<unsigned char> buf(2 * nb * c->csize);
  if (c->csize == 8) put<double>(buf, 0, cab); else put<float>(buf, 0, cab);
  yee_status st = upload(c, c->coef, buf.data(), buf.size(), s);
  if (st) return st;
  std::vector<int32_t> seg((size_t)c->px + c->d.ny + c->d.nz, 0);
  std::copy(c->segx.begin(), c->segx.end(), seg.begin());
  std::copy(c->segy.begin(), c->segy.end(), seg.begin() + c->px);
  std::copy(c->segz.begin(), c->segz.end(), seg.begin() + c->px + c->d.ny);
  if ((st = upload(c, c->segr, seg.data(), seg.size() * 4, s))) return st;
  // pageable source buffers: make sure the copies are done before they go away
  HIP_TRY(hipStreamSynchronize(s));
  return YEE_OK;
}

size_t step_lds_bytes(const yee_ctx* c, int ty, int V, int kz) {
  return yee::step_lds_bytes_for(ty, waves_per_row(c->d.nx, V), V, kz, c->csize);
}

// Kernel arguments of one step of context c at its current step count, for a
// launch shape (V samples per lane, ty rows per tile, kz planes per chunk).
// record = false: the step writes no probe samples (recomputation of steps
// already recorded).
// Cache policy of the field and CPML stores of a step with component arrays
// of comp_bytes each: streamed past the 256 MB last-level cache
// (non-temporal) when the step's field traffic -- 6 arrays read, 6 written --
// takes more than 7/8 of it (the rest holds the CPML auxiliaries and the
// tables). The written set is then evicted before the next step reads it,
// and caching it only displaces the reads; when it fits, the next step reads
// it from there and streaming the stores loses that.  Measured crossover:
// cached stores win at 194 MiB of fields, streamed ones from 238 MiB.
constexpr size_t kLastLevelCacheBytes = size_t(256) << 20;
inline bool stream_stores(size_t comp_bytes) { return 12 * comp_bytes > kLastLevelCacheBytes / 8 * 7; }

template <class T, class C>
yee::StepArgs<T, C> fill_args(const yee_ctx* c, int V, int ty, int kz, bool record = true) {
  using namespace yee;
  const auto& d = c->d;
  StepArgs<T, C> a{};
  const int cur = c->cur, nxt = cur ^ 1;
  a.fin = reinterpret_cast<const T*>(c->ws + c->fields[cur].off);
  a.fout = reinterpret_cast<T*>(c->ws + c->fields[nxt].off);
  a.cstride = c->comp_bytes / sizeof(T);
  a.pse = reinterpret_cast<C*>(c->ws + c->psi_e[c->pecur].off);
  a.pse_out = reinterpret_cast<C*>(c->ws + c->psi_e[c->pecur ^ 1].off);
  a.psbase = reinterpret_cast<const C*>(c->ws + c->psi_e[0].off);
  a.psi_span = (uint32_t)(c->psi_h[1].off + c->psi_h[1].bytes - c->psi_e[0].off);
  a.psh_in = reinterpret_cast<const C*>(c->ws + c->psi_h[cur].off);
  a.psh_out = reinterpret_cast<C*>(c->ws + c->psi_h[nxt].off);
  for (int q = 0; q < 6; ++q) a.psoff[q] = c->psi_off[q];
  a.prof = reinterpret_cast<const C*>(c->ws + c->prof.off);
  a.plen = (int32_t)c->prof_len;
  a.seg = reinterpret_cast<const int32_t*>(c->ws + c->segr.off);
  a.coef = reinterpret_cast<const Coef2<C>*>(c->ws + c->coef.off);
  a.nsx = c->nsx;
  a.nsxy = c->nsx * c->nsy;
  a.pec_plane = reinterpret_cast<const int32_t*>(c->ws + c->pecplane.off);
  a.pec_mask = reinterpret_cast<const uint8_t*>(c->ws + c->pecmask.off);
  a.rowflag = reinterpret_cast<const uint8_t*>(c->ws + c->rowflag.off);
  a.probe = reinterpret_cast<const int4*>(c->ws + c->prober.off);
  a.series = reinterpret_cast<double*>(c->ws + c->series.off);
  a.nprobe = record ? (int32_t)c->probes.size() : 0;
  a.series_slot = (int32_t)(c->n % d.series_len);
  a.series_slot2 = (int32_t)((c->n + 1) % d.series_len);
  a.src = reinterpret_cast<const SrcDev*>(c->ws + c->srcr.off);
  a.nsrc = (int32_t)c->src.size();
  a.n = c->n;
  a.dt = c->dt;
  a.nx = d.nx; a.ny = d.ny; a.nz = d.nz; a.px = c->px;
  for (int q = 0; q < 3; ++q) a.L[q] = d.cpml_cells[q];
  a.inv_d[0] = static_cast<C>(1.0 / d.dx);
  a.inv_d[1] = static_cast<C>(1.0 / d.dy);
  a.inv_d[2] = static_cast<C>(1.0 / d.dz);
  a.dt_mu = static_cast<C>(c->dt / kMu0);
  for (int q = 0; q < 6; ++q) {
    const int e = d.precision == YEE_F16S ? d.fp16_exp[q] : 0;
    a.enc[q] = std::ldexp(1.0f, e);
    a.dec[q] = std::ldexp(1.0f, -e);
  }
  a.ty = ty;
  a.kz = kz;
  a.wpr = waves_per_row(d.nx, V);
  a.ny_tiles = (d.ny + ty - 1) / ty;
  a.ntiles = a.ny_tiles * ((d.nz + kz - 1) / kz);

  a.psi_bytes = (uint32_t)c->psi_e[0].bytes;
  a.coef_bytes = (uint32_t)c->coef.bytes;
  return a;
}

// E^{n+1} of a box written by the step itself (adjoint history): the box
// {i0, i1, j0, j1, k0, k1}, the destination of component 0 and the component
// stride in elements.
struct HistOut {
  const int32_t* box;
  void* dst;
  uint64_t stride;
};

template <class T, class C, int V>
yee_status launch_step(yee_ctx* c, hipStream_t s, bool record, const HistOut* hist) {
  using namespace yee;
  StepArgs<T, C> a = fill_args<T, C>(c, V, c->ty, c->kz, record);
  const int grid = ((a.ntiles + 7) / 8) * 8;
  const int waves = (c->ty + 1) * a.wpr;
  if (waves > max_block_waves(V))
    return fail(YEE_EINVAL, "tile of %d rows x %d waves per row exceeds %d waves", c->ty, a.wpr, max_block_waves(V));
  const size_t lds = step_lds_bytes(c, c->ty, V, c->kz);
  if (lds > c->lds_limit) return fail(YEE_EINVAL, "tile of %d rows needs %zu bytes of LDS (limit %zu)", c->ty, lds, c->lds_limit);
  if constexpr (std::is_same<T, C>::value) {
    if (hist) {
      a.hist = static_cast<T*>(hist->dst);
      a.hstride = hist->stride;
      for (int q = 0; q < 6; ++q) a.hbox[q] = hist->box[q];
      hipLaunchKernelGGL((step_kernel<T, C, V, kHistory>), dim3(grid), dim3(kWave * waves), lds, s, a);
      HIP_TRY(hipGetLastError());
      return YEE_OK;
    }
  }
  if (c->dbg_count) {
    a.wcount = c->dbg_count;
    hipLaunchKernelGGL((step_kernel<T, C, V, kWriteCount>), dim3(grid), dim3(kWave * waves), lds, s, a);
    HIP_TRY(hipGetLastError());
    return YEE_OK;
  }
  if (stream_stores(c->comp_bytes))
    hipLaunchKernelGGL((step_kernel<T, C, V, kStream>), dim3(grid), dim3(kWave * waves), lds, s, a);
  else
    hipLaunchKernelGGL((step_kernel<T, C, V>), dim3(grid), dim3(kWave * waves), lds, s, a);
  HIP_TRY(hipGetLastError());
  return YEE_OK;
}

template <class T, class C>
yee_status launch_step_v(yee_ctx* c, hipStream_t s, bool record, const HistOut* hist) {
  switch (c->V) {
    case 1: return launch_step<T, C, 1>(c, s, record, hist);
    case 2: return launch_step<T, C, 2>(c, s, record, hist);
    default: return launch_step<T, C, 4>(c, s, record, hist);
  }
}

// One single step; hist (FP64 and FP32 contexts only) also writes E^{n+1} of a box.
yee_status launch_one_step(yee_ctx* c, hipStream_t s, bool record = true, const HistOut* hist = nullptr) {
  switch (c->d.precision) {
    case YEE_F64: return launch_step_v<double, double>(c, s, record, hist);
    case YEE_F32: return launch_step_v<float, float>(c, s, record, hist);
    default:
      if (hist) return fail(YEE_EINVAL, "box history is written for FP64 and FP32 contexts only");
      return launch_step_v<_Float16, float>(c, s, record, nullptr);
  }
}

// ---------------------------------------------------------------------------
// Two steps per sweep (yee_tb.hpp): FP32 arithmetic (FP32 or FP16 storage),
// rows of at most 256 samples (one wave per row).
// ---------------------------------------------------------------------------
constexpr int kTbMaxRow = 4 * yee::kWave;

size_t tb_lds_bytes(const yee_ctx* c, int ty, int V, int kz) {
  return yee::tb_lds_bytes_for(ty, V, c->tb_wpr, kz, c->d.cpml_cells[0]);
}

// Most tile rows of a two-step workgroup (ty + 3 rows of wpr waves each).
int tb_max_rows(int V, int wpr) { return yee::tb_block_waves(V) / wpr - 3; }

template <class T, class C, int V, int WPR>
yee_status launch_tb(yee_ctx* c, hipStream_t s, bool record) {
  using namespace yee;
  const StepArgs<T, C> a = fill_args<T, C>(c, V, c->tb_ty, c->tb_kz, record);
  const int grid = ((a.ntiles + 7) / 8) * 8;
  const size_t lds = tb_lds_bytes(c, c->tb_ty, V, c->tb_kz);
  if (lds > c->lds_limit) return fail(YEE_EINVAL, "two-step tile needs %zu bytes of LDS (limit %zu)", lds, c->lds_limit);
  if (c->tb_ty < 1 || c->tb_ty > tb_max_rows(V, WPR))
    return fail(YEE_EINVAL, "two-step tile of %d rows exceeds the workgroup", c->tb_ty);
  const dim3 block(kWave * WPR * (c->tb_ty + 3));
  if (stream_stores(c->comp_bytes))
    hipLaunchKernelGGL((tb_kernel<T, C, V, WPR, true>), dim3(grid), block, lds, s, a);
  else
    hipLaunchKernelGGL((tb_kernel<T, C, V, WPR>), dim3(grid), block, lds, s, a);
  HIP_TRY(hipGetLastError());
  return YEE_OK;
}

// rows of at most 64, 128 and 256 samples: one wave of one or two samples per
// lane, or two waves of two
template <class T>
yee_status launch_tb_v(yee_ctx* c, hipStream_t s, bool record) {
  if (c->tb_V == 1) return launch_tb<T, float, 1, 1>(c, s, record);
  if (c->tb_wpr == 1) return launch_tb<T, float, 2, 1>(c, s, record);
  return launch_tb<T, float, 2, 2>(c, s, record);
}

yee_status launch_two_steps(yee_ctx* c, hipStream_t s, bool record = true) {
  return c->d.precision == YEE_F32 ? launch_tb_v<float>(c, s, record) : launch_tb_v<_Float16>(c, s, record);
}

yee_status fold_dft(yee_ctx* c, hipStream_t s) {
  const int64_t count = c->n - c->folded;
  if (count <= 0) return YEE_OK;
  const int np = (int)c->probes.size(), nf = (int)c->freqs.size();
  if (np > 0 && nf > 0) {
    const int waves = np * nf;
    const int blocks = (waves * yee::kWave + 255) / 256;
    hipLaunchKernelGGL(yee::dft_fold_kernel, dim3(blocks), dim3(256), 0, s,
                       reinterpret_cast<const double*>(c->ws + c->series.off), np, c->d.series_len,
                       c->folded + 1, (int)count, reinterpret_cast<const double*>(c->ws + c->freqr.off),
                       nf, c->dt, reinterpret_cast<double2*>(c->ws + c->dft.off),
                       reinterpret_cast<uint32_t*>(c->ws + c->stat.off));
    HIP_TRY(hipGetLastError());
  }
  c->folded = c->n;
  return YEE_OK;
}

constexpr int kMinChunk = 8;   // fewest planes per chunk of the automatic launch above 2^20 cells
// most planes per chunk of the automatic launch: where one round would take
// longer chunks (one workgroup per CU), several rounds of 64-plane chunks run
// faster (512 x 512 x 256 per step: FP16 storage 0.673 -> 0.620 ms, FP32
// 0.884 -> 0.825 ms)
constexpr int kMaxChunk = 64;

// Workgroups of the step kernel that fit one CU at once.
template <class T, class C, int V>
int step_blocks_per_cu(int threads, size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, yee::step_kernel<T, C, V>, threads, lds) != hipSuccess) n = 1;
  return std::max(1, n);
}

template <class T, class C>
int step_blocks_per_cu_v(int V, int threads, size_t lds) {
  switch (V) {
    case 1: return step_blocks_per_cu<T, C, 1>(threads, lds);
    case 2: return step_blocks_per_cu<T, C, 2>(threads, lds);
    default: return step_blocks_per_cu<T, C, 4>(threads, lds);
  }
}

int step_slots(const yee_ctx* c, int threads, size_t lds) {
  int dev_id = 0, cus = 0;
  if (hipGetDevice(&dev_id) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id) != hipSuccess || cus < 1)
    cus = 1;
  int per_cu = 1;
  switch (c->d.precision) {
    case YEE_F64: per_cu = step_blocks_per_cu_v<double, double>(c->V, threads, lds); break;
    case YEE_F32: per_cu = step_blocks_per_cu_v<float, float>(c->V, threads, lds); break;
    default: per_cu = step_blocks_per_cu_v<_Float16, float>(c->V, threads, lds); break;
  }
  return per_cu * cus;
}

// Samples per lane: one while a row fits in four waves; wider rows (up to
// eight waves) keep one sample per lane in FP32 and take two otherwise (with
// 2-byte storage one-sample loads would be half-width).  Measured at
// 512 x 512 x 256: FP32 1.04 ms per step with one sample, 1.35 with two;
// FP16 storage 1.08 with two, 1.10 with one.
// Samples per lane when the caller does not choose: one up to 256-sample rows;
// past that two for FP32 and FP16 storage (512 x 512 x 256: 0.88 against
// 1.10 ms in FP32, 0.69 against 1.01 ms in FP16 storage), but one for FP64,
// whose two-sample kernel spills (300 x 256 x 128: 0.43 against 1.10 ms).
int default_samples_per_lane(const yee_grid_desc& d) {
  return (d.nx <= 4 * yee::kWave || d.precision == YEE_F64) ? 1 : 2;
}

// Workgroups of the two-step kernel that fit one CU at once.
template <class T, int V, int WPR>
int tb_blocks_per_cu(int threads, size_t lds) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, yee::tb_kernel<T, float, V, WPR>, threads, lds) != hipSuccess)
    n = 1;
  return std::max(1, n);
}

int tb_slots(const yee_ctx* c, int threads, size_t lds) {
  int dev_id = 0, cus = 0;
  if (hipGetDevice(&dev_id) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id) != hipSuccess || cus < 1)
    cus = 1;
  int per_cu = 1;
  const bool f32 = c->d.precision == YEE_F32;
  if (c->tb_V == 1) per_cu = f32 ? tb_blocks_per_cu<float, 1, 1>(threads, lds) : tb_blocks_per_cu<_Float16, 1, 1>(threads, lds);
  else if (c->tb_wpr == 1) per_cu = f32 ? tb_blocks_per_cu<float, 2, 1>(threads, lds) : tb_blocks_per_cu<_Float16, 2, 1>(threads, lds);
  else per_cu = f32 ? tb_blocks_per_cu<float, 2, 2>(threads, lds) : tb_blocks_per_cu<_Float16, 2, 2>(threads, lds);
  return per_cu * cus;
}

// Whether yee_step advances two steps per sweep, and its launch shape.  The
// sweep takes FP32 arithmetic (FP32 or FP16 storage) and rows of at most 256
// samples; with probes the ring must hold both steps.  Tile rows: the count
// whose tiles, with chunks sized so that every tile is resident at once, do
// the least work per workgroup (a tile computes 4 ty + 6 row-stages on each of
// kz + 3 planes); for 256^3 that is four rows, 64 y-tiles of 64-plane chunks,
// one workgroup per CU.
// Whether the automatic mode (steps_per_sweep 0) takes two-step sweeps.
constexpr bool kTbAutomatic = false;

void tb_default_launch(yee_ctx* c) {
  const auto& d = c->d;
  c->tb_ok = false;
  if (c->tb_req == 1 || (c->tb_req == 0 && !kTbAutomatic)) return;
  if (d.precision == YEE_F64 || d.nx > kTbMaxRow || (!c->probes.empty() && d.series_len < 2)) return;
  c->tb_V = d.nx <= yee::kWave ? 1 : 2;
  c->tb_wpr = d.nx <= 2 * yee::kWave ? 1 : 2;
  const int64_t cells = (int64_t)d.nx * d.ny * d.nz;
  const int min_chunk = cells <= (int64_t(1) << 18) ? 2 : (cells <= (int64_t(1) << 20) ? 4 : kMinChunk);
  const int tymax = std::min(tb_max_rows(c->tb_V, c->tb_wpr), d.ny);
  int best_ty = 0, best_kz = 0;
  double best = 0.0;
  for (int ty = (c->tb_ty_req ? c->tb_ty_req : 1); ty <= (c->tb_ty_req ? c->tb_ty_req : tymax); ++ty) {
    const int ny_tiles = (d.ny + ty - 1) / ty;
    int kz;
    int slots = 1;
    if (c->tb_kz_req > 0) {
      kz = std::min(c->tb_kz_req, d.nz);
    } else {
      slots = tb_slots(c, (ty + 3) * c->tb_wpr * yee::kWave, tb_lds_bytes(c, ty, c->tb_V, d.nz));
      const int chunks = std::max(1, slots / ny_tiles);
      kz = std::min(d.nz, std::max(min_chunk, (d.nz + chunks - 1) / chunks));
    }
    if (tb_lds_bytes(c, ty, c->tb_V, kz) > c->lds_limit) continue;
    if (c->tb_kz_req == 0) {
      // a tile's work times the tiles each CU runs (resident workgroups share
      // their CU, so a CU's work is what counts)
      int dev_id = 0, cus = 1;
      if (hipGetDevice(&dev_id) != hipSuccess ||
          hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id) != hipSuccess || cus < 1)
        cus = 1;
      const int64_t tiles = (int64_t)ny_tiles * ((d.nz + kz - 1) / kz);
      const double per_cu = (double)((tiles + cus - 1) / cus);
      const double cost = per_cu * (4.0 * ty + 6.0) * (std::min(kz, d.nz) + 3.0);
      if (best_ty == 0 || cost < best) { best = cost; best_ty = ty; best_kz = kz; }
    } else if (best_ty == 0) {
      best_ty = ty;
      best_kz = kz;
    }
  }
  if (best_ty == 0) return;
  c->tb_ty = best_ty;
  c->tb_kz = best_kz;
  c->tb_ok = true;
}

void default_launch(yee_ctx* c) {
  const auto& d = c->d;
  c->V = c->vpl ? c->vpl : default_samples_per_lane(d);
  const int wpr = waves_per_row(d.nx, c->V);
  // Small grids: a step's time is the march of one chunk (its planes run one
  // after another), not bandwidth, so they take shorter chunks and, up to
  // 2^18 cells, at most two rows per tile, for more workgroups in flight.
  // Measured per step: 12 x 12 x 140 16.8 -> 8.9 us, 32^3 21.1 -> 10.0 us,
  // 64^3 21.6 -> 12.6 us (two rows, two-plane chunks); 96^3 25.7 -> 22.4 us
  // (four-plane chunks; two-plane chunks were slower there, 37.8 us).
  const int64_t cells = (int64_t)d.nx * d.ny * d.nz;
  const bool tiny = cells <= (int64_t(1) << 18);
  const int min_chunk = tiny ? 2 : (cells <= (int64_t(1) << 20) ? 4 : kMinChunk);
  // rows per tile: workgroups of at most 12 waves, so that two fit a CU, and
  // within the kernel's wave limit for V samples per lane; measured best for
  // the 256^3 grid: two rows of four waves plus the halo row; for rows of two
  // waves four rows, not five (96^3: 22.6 against 22.9 us per step, 128^3:
  // 30.7 against 32.4 us)
  c->ty = c->ty_req ? c->ty_req
                    : std::max(1, std::min({tiny ? 2 : (wpr == 2 ? 4 : 7), d.ny, 12 / wpr - 1,
                                            yee::max_block_waves(c->V) / wpr - 1}));
  for (;;) {
    if (c->kz_req > 0) {
      c->kz = std::min(c->kz_req, d.nz);
    } else {
      // planes per chunk: the fewest (at least min_chunk) that let every
      // tile be resident at once, so the launch runs in one round and each
      // chunk pays its warm-up plane once over as long a march as possible
      const int threads = (c->ty + 1) * wpr * yee::kWave;
      const int slots = step_slots(c, threads, step_lds_bytes(c, c->ty, c->V, d.nz));
      const int ny_tiles = (d.ny + c->ty - 1) / c->ty;
      const int chunks = std::max(1, slots / ny_tiles);
      c->kz = std::min({d.nz, kMaxChunk, std::max(min_chunk, (d.nz + chunks - 1) / chunks)});
    }
    // keep the LDS rows and z tables within the device's per-workgroup limit
    if (c->ty == 1 || step_lds_bytes(c, c->ty, c->V, c->kz) <= c->lds_limit) break;
    --c->ty;
  }
  tb_default_launch(c);
}

template <class T>
void host_to_storage(const double* in, std::vector<unsigned char>& out, const yee_grid_desc& d,
                     int px, float enc) {
  T* o = reinterpret_cast<T*>(out.data());
  for (size_t k = 0; k < (size_t)d.nz; ++k)
    for (size_t j = 0; j < (size_t)d.ny; ++j)
      for (size_t i = 0; i < (size_t)d.nx; ++i)
        o[(k * d.ny + j) * px + i] = static_cast<T>(static_cast<float>(in[(k * d.ny + j) * d.nx + i]) * enc);
}

// ---------------------------------------------------------------------------
// Batched stepper (serving): contexts of one storage precision share one
// fixed-size launch: FP32 and FP64 at one sample per lane (rows of at most
// 256 samples), FP16 storage at two (rows of at most 512: 4-byte row loads).
// ---------------------------------------------------------------------------
#ifndef YEE_BATCH_WAVES
#define YEE_BATCH_WAVES 12
#endif
constexpr int kBatchBlockWaves = YEE_BATCH_WAVES;  // waves per workgroup of the batched launch
constexpr int kBatchMaxChunk = 32;    // most planes per z-chunk of a batched grid
constexpr int kBatchMinChunk = 2;     // fewest: with few requests running, short marches keep a step short
int batch_V(int prec) { return prec == YEE_F16S ? 2 : 1; }

// bytes of one slot descriptor in the device table (the largest of the
// precisions, so the table's size does not depend on the precision)
size_t batch_desc_bytes() {
  return std::max({sizeof(yee::SlotDesc<float, float>), sizeof(yee::SlotDesc<_Float16, float>),
                   sizeof(yee::SlotDesc<double, double>)});
}

int batch_tile_rows(const yee_ctx* c, int V) {
  const int wpr = waves_per_row(c->d.nx, V);
  return std::max(1, std::min(c->d.ny, kBatchBlockWaves / wpr - 1));
}

size_t batch_lds_bytes(int prec) {
  const int V = batch_V(prec);
  const size_t csize = prec == YEE_F64 ? sizeof(double) : sizeof(float);
  size_t m = 0;
  for (int wpr = 1; wpr <= 4; ++wpr) {
    const int ty = std::max(1, kBatchBlockWaves / wpr - 1);
    m = std::max(m, yee::step_lds_bytes_for(ty, wpr, V, kBatchMaxChunk, csize));
  }
  return m;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
namespace {

// The mask of z-plane k ([ny][px] bytes), added (all clear) on first use.
std::vector<uint8_t>& pec_plane_mask(yee_ctx* c, int k) {
  auto it = std::find(c->pec_k.begin(), c->pec_k.end(), k);
  if (it != c->pec_k.end()) return c->pec_masks[(size_t)(it - c->pec_k.begin())];
  c->pec_k.push_back(k);
  c->pec_masks.emplace_back((size_t)c->d.ny * c->px, (uint8_t)0);
  return c->pec_masks.back();
}

}  // namespace

namespace {

constexpr int64_t kStateMagic = 0x3154415453454559LL;   // "YEESTAT1"
constexpr int kStateWords = 32;                         // header: 32 int64 (256 bytes)
constexpr int kStateShapeWords = 22;                    // words that must match on load

struct StateLayout {
  size_t fields, pse, psh, series, dft, stat, total;
};

StateLayout state_layout(const yee_ctx* c) {
  StateLayout L{};
  size_t off = kStateWords * sizeof(int64_t);
  auto take = [&](size_t& at, size_t bytes) {
    at = off;
    off += align256(bytes);
  };
  take(L.fields, 6 * c->comp_bytes);
  take(L.pse, c->psi_e[0].bytes);
  take(L.psh, c->psi_h[0].bytes);
  take(L.series, c->series.bytes);
  take(L.dft, c->dft.bytes);
  take(L.stat, c->stat.bytes);
  L.total = off;
  return L;
}

// Header words: 0..21 describe the shape of the state, 24 and 25 the step
// and fold counters.
void state_words(const yee_ctx* c, int64_t w[kStateWords]) {
  const auto& d = c->d;
  std::fill(w, w + kStateWords, int64_t(0));
  w[0] = kStateMagic;
  w[1] = YEE_API_VERSION;
  w[2] = d.nx; w[3] = d.ny; w[4] = d.nz;
  w[5] = c->px;
  w[6] = d.precision;
  for (int q = 0; q < 3; ++q) w[7 + q] = d.cpml_cells[q];
  for (int q = 0; q < 6; ++q) w[10 + q] = d.precision == YEE_F16S ? d.fp16_exp[q] : 0;
  w[16] = (int64_t)c->probes.size();
  w[17] = (int64_t)c->freqs.size();
  w[18] = d.series_len;
  w[19] = (int64_t)c->comp_bytes;
  w[20] = (int64_t)c->psi_e[0].bytes;
  w[21] = (int64_t)state_layout(c).total;
  w[24] = c->n;
  w[25] = c->folded;
}

}  // namespace

extern "C" {

const char* yee_last_error(void) { return g_err.c_str(); }
int32_t yee_api_version(void) { return YEE_API_VERSION; }

yee_status yee_create(const yee_grid_desc* desc, yee_ctx** out) {
  if (!out) return fail(YEE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!desc) return fail(YEE_EINVAL, "desc is NULL");
  const yee_grid_desc& d = *desc;
  if (d.nx < 2 || d.ny < 2 || d.nz < 2) return fail(YEE_EINVAL, "grid must have >= 2 cells per axis");
  if (d.precision < YEE_F64 || d.precision > YEE_F16S) return fail(YEE_EINVAL, "bad precision %d", d.precision);
  if (!(d.dx > 0) || !(d.dy > 0) || !(d.dz > 0)) return fail(YEE_EINVAL, "cell sizes must be > 0");
  if (!(d.courant > 0.0) || d.courant > 1.0) return fail(YEE_EINVAL, "Courant number %g not in (0, 1]", d.courant);
  if (d.series_len < 1) return fail(YEE_EINVAL, "series_len must be >= 1");
  const int n3[3] = {d.nx, d.ny, d.nz};
  for (int q = 0; q < 3; ++q)
    if (d.cpml_cells[q] < 0 || 2 * d.cpml_cells[q] > n3[q])
      return fail(YEE_EINVAL, "CPML thickness %d invalid for axis of %d cells", d.cpml_cells[q], n3[q]);
  if (d.cpml_m < 0 || d.cpml_kappa_max < 1.0 || d.cpml_alpha_max < 0)
    return fail(YEE_EINVAL, "CPML grading parameters out of range");
  for (int q = 0; q < 6; ++q)
    if (d.fp16_exp[q] < -30 || d.fp16_exp[q] > 30) return fail(YEE_EINVAL, "fp16 exponent out of range");
  auto* c = new (std::nothrow) yee_ctx();
  if (!c) return fail(YEE_ENOMEM, "host allocation failed");
  c->d = d;
  if (d.nx > kMaxRow) {
    delete c;
    return fail(YEE_EINVAL, "nx = %d exceeds the row limit (%d)", d.nx, kMaxRow);
  }
  c->tsize = storage_size(d.precision);
  c->csize = compute_size(d.precision);
  // x pitch: a whole number of 128-byte lines (and of the widest lane vector)
  const int line = std::max(128 / (int)c->tsize, 4);
  c->px = ((d.nx + line - 1) / line) * line;
  if ((uint64_t)d.nz * d.ny * c->px >= (1ull << 31)) {
    delete c;
    return fail(YEE_EINVAL, "grid too large for 32-bit element offsets");
  }
  // the step addresses a field set (six components) and the psi regions with
  // 32-bit byte offsets
  if (6 * ((uint64_t)(d.nz + 1) * d.ny * c->px * c->tsize + 256) >= (1ull << 31)) {
    delete c;
    return fail(YEE_EINVAL, "grid too large: a set of six components must stay below 2 GiB");
  }
  // ... and the four CPML auxiliary regions (E and H side, two sets each, laid
  // out consecutively) under one resource whose out-of-range marker is 2^31:
  // their total must stay below it
  {
    size_t pl[6];
    psi_lengths(c, pl);
    const uint64_t psib = align256((2 * (pl[0] + pl[1] + pl[3])) * c->csize);
    if (4 * psib >= (1ull << 31)) {
      delete c;
      return fail(YEE_EINVAL, "CPML layers too thick: the four auxiliary regions (%llu bytes) must stay below 2 GiB",
                  (unsigned long long)(4 * psib));
    }
  }
  c->dt = d.courant / (kC0 * std::sqrt(1.0 / (d.dx * d.dx) + 1.0 / (d.dy * d.dy) + 1.0 / (d.dz * d.dz)));
  c->segx.assign(d.nx, 0);
  c->segy.assign(d.ny, 0);
  c->segz.assign(d.nz, 0);
  c->eps.assign(1, 1.0);
  c->sig.assign(1, 0.0);
  *out = c;
  return YEE_OK;
}

void yee_destroy(yee_ctx* ctx) { delete ctx; }

yee_status yee_time_step(const yee_ctx* c, double* dt) {
  if (!c || !dt) return fail(YEE_EINVAL, "NULL argument");
  *dt = c->dt;
  return YEE_OK;
}

yee_status yee_set_materials(yee_ctx* c, int32_t nsx, int32_t nsy, int32_t nsz, const int32_t* seg_x,
                             const int32_t* seg_y, const int32_t* seg_z, const double* eps_r,
                             const double* sigma) {
  if (!c || !seg_x || !seg_y || !seg_z || !eps_r || !sigma) return fail(YEE_EINVAL, "NULL argument");
  if (nsx < 1 || nsy < 1 || nsz < 1) return fail(YEE_EINVAL, "lattice must have >= 1 block per axis");
  if (c->bound && (nsx != c->nsx || nsy != c->nsy || nsz != c->nsz))
    return fail(YEE_ESTATE, "lattice shape is fixed once the workspace is bound");
  const auto& d = c->d;
  for (int i = 0; i < d.nx; ++i) if (seg_x[i] < 0 || seg_x[i] >= nsx) return fail(YEE_EINVAL, "seg_x[%d] out of range", i);
  for (int i = 0; i < d.ny; ++i) if (seg_y[i] < 0 || seg_y[i] >= nsy) return fail(YEE_EINVAL, "seg_y[%d] out of range", i);
  for (int i = 0; i < d.nz; ++i) if (seg_z[i] < 0 || seg_z[i] >= nsz) return fail(YEE_EINVAL, "seg_z[%d] out of range", i);
  const size_t nb = (size_t)nsx * nsy * nsz;
  for (size_t b = 0; b < nb; ++b)
    if (!(eps_r[b] >= 1e-3) || !(sigma[b] >= 0.0) || !std::isfinite(eps_r[b]) || !std::isfinite(sigma[b]))
      return fail(YEE_EINVAL, "material %zu out of range (eps_r %g, sigma %g)", b, eps_r[b], sigma[b]);
  c->nsx = nsx; c->nsy = nsy; c->nsz = nsz;
  c->segx.assign(seg_x, seg_x + d.nx);
  c->segy.assign(seg_y, seg_y + d.ny);
  c->segz.assign(seg_z, seg_z + d.nz);
  c->eps.assign(eps_r, eps_r + nb);
  c->sig.assign(sigma, sigma + nb);
  return YEE_OK;
}

yee_status yee_upload_materials(yee_ctx* c, void* stream) {
  if (!c) return fail(YEE_EINVAL, "NULL context");
  if (!c->bound) return fail(YEE_ESTATE, "no workspace bound");
  return upload_materials_impl(c, (hipStream_t)stream);
}


yee_status yee_add_pec_plane(yee_ctx* c, int32_t k, const uint8_t* mask) {
  if (!c || !mask) return fail(YEE_EINVAL, "NULL argument");
  if (c->bound) return fail(YEE_ESTATE, "configuration is frozen once the workspace is bound");
  if (k <= 0 || k >= c->d.nz) return fail(YEE_EINVAL, "PEC plane k = %d not in (0, nz)", k);
  std::vector<uint8_t>& m = pec_plane_mask(c, k);
  for (int j = 0; j < c->d.ny; ++j)
    for (int i = 0; i < c->d.nx; ++i) m[(size_t)j * c->px + i] |= mask[(size_t)j * c->d.nx + i] & 7;
  return YEE_OK;
}

yee_status yee_set_pec_mask(yee_ctx* c, const uint8_t* mask) {
  if (!c || !mask) return fail(YEE_EINVAL, "NULL argument");
  if (c->bound) return fail(YEE_ESTATE, "configuration is frozen once the workspace is bound");
  const auto& d = c->d;
  const size_t plane = (size_t)d.nx * d.ny;
  for (size_t q = 0; q < plane * d.nz; ++q)
    if (mask[q] & ~7u) return fail(YEE_EINVAL, "mask byte %zu has bits other than 0..2 set", q);
  // one plane mask per z-plane that holds a set bit, merged with planes
  // already given by yee_add_pec_plane
  for (int k = 0; k < d.nz; ++k) {
    const uint8_t* mk = mask + (size_t)k * plane;
    if (std::all_of(mk, mk + plane, [](uint8_t v) { return v == 0; })) continue;
    std::vector<uint8_t>& m = pec_plane_mask(c, k);
    for (int j = 0; j < d.ny; ++j)
      for (int i = 0; i < d.nx; ++i) m[(size_t)j * c->px + i] |= mk[(size_t)j * d.nx + i];
  }
  return YEE_OK;
}

yee_status yee_add_source(yee_ctx* c, const yee_source* s) {
  if (!c || !s) return fail(YEE_EINVAL, "NULL argument");
  if (c->bound) return fail(YEE_ESTATE, "configuration is frozen once the workspace is bound");
  const auto& d = c->d;
  if (s->component < 0 || s->component > 2) return fail(YEE_EINVAL, "source component must be an E component");
  if (s->i < 0 || s->i >= d.nx || s->j < 0 || s->j >= d.ny || s->k < 0 || s->k >= d.nz)
    return fail(YEE_EINVAL, "source (%d,%d,%d) outside the grid", s->i, s->j, s->k);
  if (s->waveform != YEE_GAUSS_DERIV && s->waveform != YEE_MOD_GAUSS) return fail(YEE_EINVAL, "bad waveform");
  if (!(s->tau > 0)) return fail(YEE_EINVAL, "tau must be > 0");
  if ((int)c->src.size() >= yee::kMaxSources) return fail(YEE_EINVAL, "at most %d sources", yee::kMaxSources);
  yee::SrcDev sd{};
  sd.comp = s->component; sd.i = s->i; sd.j = s->j; sd.k = s->k; sd.kind = s->waveform;
  sd.amp = s->amp; sd.t0 = s->t0; sd.tau = s->tau; sd.f0 = s->f0;
  c->src.push_back(sd);
  return YEE_OK;
}

yee_status yee_add_probe(yee_ctx* c, int32_t comp, int32_t i, int32_t j, int32_t k, int32_t* id) {
  if (!c) return fail(YEE_EINVAL, "NULL context");
  if (c->bound) return fail(YEE_ESTATE, "configuration is frozen once the workspace is bound");
  const auto& d = c->d;
  if (comp < 0 || comp > 5) return fail(YEE_EINVAL, "probe component %d not in 0..5", comp);
  if (i < 0 || i >= d.nx || j < 0 || j >= d.ny || k < 0 || k >= d.nz)
    return fail(YEE_EINVAL, "probe (%d,%d,%d) outside the grid", i, j, k);
  c->probes.push_back(int4{comp, i, j, k});
  if (id) *id = (int32_t)c->probes.size() - 1;
  return YEE_OK;
}

yee_status yee_set_dft_freqs(yee_ctx* c, const double* freqs, int32_t nf) {
  if (!c || (nf > 0 && !freqs) || nf < 0) return fail(YEE_EINVAL, "bad argument");
  if (c->bound) return fail(YEE_ESTATE, "configuration is frozen once the workspace is bound");
  c->freqs.assign(freqs, freqs + nf);
  return YEE_OK;
}

yee_status yee_footprint(const yee_ctx* c, int64_t* bytes) {
  if (!c || !bytes) return fail(YEE_EINVAL, "NULL argument");
  yee_ctx tmp = *c;
  layout(&tmp);
  *bytes = tmp.ws_bytes;
  return YEE_OK;
}

yee_status yee_bind_workspace(yee_ctx* c, void* dev, int64_t bytes) {
  if (!c || !dev) return fail(YEE_EINVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(dev) & 255) return fail(YEE_EINVAL, "workspace must be 256-byte aligned");
  layout(c);
  if (bytes < c->ws_bytes) return fail(YEE_ENOMEM, "workspace has %lld bytes, needs %lld", (long long)bytes, (long long)c->ws_bytes);
  int dev_id = 0, lds = 0;
  HIP_TRY(hipGetDevice(&dev_id));
  HIP_TRY(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev_id));
  if (lds > 0) c->lds_limit = (size_t)lds;
  c->ws = static_cast<unsigned char*>(dev);
  c->bound = true;
  default_launch(c);
  return YEE_OK;
}

yee_status yee_set_launch(yee_ctx* c, int32_t tile_rows, int32_t chunk_planes, int32_t samples_per_lane) {
  if (!c) return fail(YEE_EINVAL, "NULL context");
  if (samples_per_lane != 0 && samples_per_lane != 1 && samples_per_lane != 2 && samples_per_lane != 4)
    return fail(YEE_EINVAL, "samples_per_lane must be 0, 1, 2 or 4");
  const int V = samples_per_lane ? samples_per_lane : default_samples_per_lane(c->d);
  const int wpr = waves_per_row(c->d.nx, V);
  if (wpr + 1 > 2 * yee::max_block_waves(V) || (wpr * 2 > yee::max_block_waves(V)))
    return fail(YEE_EINVAL, "rows of %d samples need %d waves at %d samples per lane: too many", c->d.nx, wpr, V);
  if (tile_rows < 0 || chunk_planes < 0 || (tile_rows > 0 && (tile_rows + 1) * wpr > yee::max_block_waves(V)))
    return fail(YEE_EINVAL, "tile_rows %d with %d waves per row exceeds %d waves per workgroup", tile_rows, wpr,
                yee::max_block_waves(V));
  c->ty_req = tile_rows;
  c->kz_req = chunk_planes;
  c->vpl = samples_per_lane;
  if (c->bound) default_launch(c);   // host state only: steps already queued keep their arguments
  return YEE_OK;
}

yee_status yee_set_time_blocking(yee_ctx* c, int32_t steps_per_sweep, int32_t tile_rows, int32_t chunk_planes) {
  if (!c) return fail(YEE_EINVAL, "NULL context");
  if (steps_per_sweep < 0 || steps_per_sweep > 2) return fail(YEE_EINVAL, "steps_per_sweep must be 0, 1 or 2");
  const int tb_wpr = c->d.nx <= 2 * yee::kWave ? 1 : 2;
  const int tb_rows = tb_max_rows(c->d.nx <= yee::kWave ? 1 : 2, tb_wpr);
  if (tile_rows < 0 || tile_rows > tb_rows || chunk_planes < 0)
    return fail(YEE_EINVAL, "tile_rows must be 0..%d for rows of %d samples, chunk_planes >= 0", tb_rows, c->d.nx);
  const auto& d = c->d;
  if (steps_per_sweep == 2 && (d.precision == YEE_F64 || d.nx > kTbMaxRow))
    return fail(YEE_EINVAL, "two steps per sweep take FP32 or FP16 storage and rows of at most %d samples", kTbMaxRow);
  if (steps_per_sweep == 2 && !c->probes.empty() && d.series_len < 2)
    return fail(YEE_EINVAL, "two steps per sweep need a probe ring of at least 2 steps");
  c->tb_req = steps_per_sweep;
  c->tb_ty_req = tile_rows;
  c->tb_kz_req = chunk_planes;
  if (c->bound) {
    tb_default_launch(c);
    if (steps_per_sweep == 2 && !c->tb_ok) return fail(YEE_EINVAL, "the two-step tile does not fit the device's LDS");
  }
  return YEE_OK;
}

yee_status yee_launch_info(const yee_ctx* c, int32_t* steps_per_sweep, int32_t* tile_rows, int32_t* chunk_planes,
                           int32_t* samples_per_lane) {
  if (!c || !steps_per_sweep || !tile_rows || !chunk_planes || !samples_per_lane) return fail(YEE_EINVAL, "NULL argument");
  if (!c->bound) return fail(YEE_ESTATE, "no workspace bound");
  *steps_per_sweep = c->tb_ok ? 2 : 1;
  *tile_rows = c->tb_ok ? c->tb_ty : c->ty;
  *chunk_planes = c->tb_ok ? c->tb_kz : c->kz;
  *samples_per_lane = c->tb_ok ? c->tb_V : c->V;
  return YEE_OK;
}

yee_status yee_debug_layout(const yee_ctx* c, int64_t* comp_stride, int32_t* row_pitch) {
  if (!c || !comp_stride || !row_pitch) return fail(YEE_EINVAL, "NULL argument");
  *comp_stride = (int64_t)(c->comp_bytes / c->tsize);
  *row_pitch = c->px;
  return YEE_OK;
}

yee_status yee_debug_set_write_counts(yee_ctx* c, uint32_t* device_counts, int64_t n_elems) {
  if (!c) return fail(YEE_EINVAL, "NULL context");
  if (device_counts && n_elems < 6 * (int64_t)(c->comp_bytes / c->tsize))
    return fail(YEE_ENOMEM, "write counts need %lld elements, got %lld", (long long)(6 * (c->comp_bytes / c->tsize)),
                (long long)n_elems);
  c->dbg_count = device_counts;
  return YEE_OK;
}

yee_status yee_reset(yee_ctx* c, void* stream) {
  if (!c) return fail(YEE_EINVAL, "NULL context");
  if (!c->bound) return fail(YEE_ESTATE, "no workspace bound");
  hipStream_t s = (hipStream_t)stream;
  const auto& d = c->d;
  // state: both field sets, psi, series, dft, status flags (one contiguous run) -- zeroed
  const size_t state_end = c->stat.off + align256(c->stat.bytes);
  HIP_TRY(hipMemsetAsync(c->ws, 0, state_end, s));
  yee_status st = upload_materials_impl(c, s);
  if (st) return st;
  // CPML profiles
  std::vector<unsigned char> pbuf(c->prof.bytes, 0);
  const int n3[3] = {d.nx, d.ny, d.nz};
  const double dw[3] = {d.dx, d.dy, d.dz};
  for (int side = 0; side < 2; ++side)
    for (int ax = 0; ax < 3; ++ax) {
      std::vector<double> b, a, k;
      cpml_profile(d, dw[ax], c->dt, n3[ax], d.cpml_cells[ax], side, b, a, k);
      b.resize(c->prof_len, 0.0); a.resize(c->prof_len, 0.0); k.resize(c->prof_len, 1.0);
      const size_t base = ((size_t)(side * 3 + ax) * 3) * c->prof_len * c->csize;
      if (c->csize == 8) {
        put<double>(pbuf, base, b); put<double>(pbuf, base + c->prof_len * 8, a); put<double>(pbuf, base + 2 * c->prof_len * 8, k);
      } else {
        put<float>(pbuf, base, b); put<float>(pbuf, base + c->prof_len * 4, a); put<float>(pbuf, base + 2 * c->prof_len * 4, k);
      }
    }
  if ((st = upload(c, c->prof, pbuf.data(), pbuf.size(), s))) return st;
  // PEC planes
  std::vector<int32_t> plane(d.nz, -1);
  std::vector<uint8_t> masks(c->pecmask.bytes, 0);
  for (size_t p = 0; p < c->pec_k.size(); ++p) {
    plane[c->pec_k[p]] = (int32_t)p;
    std::copy(c->pec_masks[p].begin(), c->pec_masks[p].end(), masks.begin() + p * (size_t)d.ny * c->px);
  }
  if ((st = upload(c, c->pecplane, plane.data(), plane.size() * 4, s))) return st;
  if ((st = upload(c, c->pecmask, masks.data(), masks.size(), s))) return st;
  // row flags, sources, probes, frequencies
  std::vector<uint8_t> flags((size_t)d.nz * d.ny, 0);
  for (auto& sd : c->src) flags[(size_t)sd.k * d.ny + sd.j] |= 1;
  for (auto& p : c->probes) flags[(size_t)p.w * d.ny + p.z] |= 2;
  if ((st = upload(c, c->rowflag, flags.data(), flags.size(), s))) return st;
  if ((st = upload(c, c->srcr, c->src.data(), c->src.size() * sizeof(yee::SrcDev), s))) return st;
  if ((st = upload(c, c->prober, c->probes.data(), c->probes.size() * sizeof(int4), s))) return st;
  if ((st = upload(c, c->freqr, c->freqs.data(), c->freqs.size() * sizeof(double), s))) return st;
  HIP_TRY(hipStreamSynchronize(s));
  c->n = 0;
  c->folded = 0;
  c->cur = 0;
  c->pecur = 0;
  return YEE_OK;
}

yee_status yee_set_field(yee_ctx* c, int32_t comp, const double* host, void* stream) {
  if (!c || !host) return fail(YEE_EINVAL, "NULL argument");
  if (!c->bound) return fail(YEE_ESTATE, "no workspace bound");
  if (comp < 0 || comp > 5) return fail(YEE_EINVAL, "component %d not in 0..5", comp);
  const auto& d = c->d;
  std::vector<unsigned char> buf((size_t)d.nz * d.ny * c->px * c->tsize, 0);
  const float enc = d.precision == YEE_F16S ? std::ldexp(1.0f, d.fp16_exp[comp]) : 1.0f;
  if (d.precision == YEE_F64) {
    double* o = reinterpret_cast<double*>(buf.data());
    for (size_t k = 0; k < (size_t)d.nz; ++k)
      for (size_t j = 0; j < (size_t)d.ny; ++j)
        for (size_t i = 0; i < (size_t)d.nx; ++i) o[(k * d.ny + j) * c->px + i] = host[(k * d.ny + j) * d.nx + i];
  } else if (d.precision == YEE_F32) {
    host_to_storage<float>(host, buf, d, c->px, 1.0f);
  } else {
    // round from double directly to fp16 (nearest even) after exact scaling;
    // a finite value beyond the format's range is refused (NaN and infinities
    // are stored as given and reported by yee_status_flags)
    for (size_t q = 0; q < (size_t)d.nz * d.ny * d.nx; ++q)
      if (std::isfinite(host[q]) && std::fabs(host[q] * (double)enc) > 65504.0)
        return fail(YEE_EOVERFLOW, "component %d: |value x 2^%d| = %g exceeds the fp16 range (65504)", comp,
                    d.fp16_exp[comp], std::fabs(host[q] * (double)enc));
    _Float16* o = reinterpret_cast<_Float16*>(buf.data());
    for (size_t k = 0; k < (size_t)d.nz; ++k)
      for (size_t j = 0; j < (size_t)d.ny; ++j)
        for (size_t i = 0; i < (size_t)d.nx; ++i)
          o[(k * d.ny + j) * c->px + i] = static_cast<_Float16>(host[(k * d.ny + j) * d.nx + i] * (double)enc);
  }
  hipStream_t s = (hipStream_t)stream;
  const int cur = c->cur;
  HIP_TRY(hipMemcpyAsync(c->ws + c->fields[cur].off + comp * c->comp_bytes, buf.data(), buf.size(),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  return YEE_OK;
}

yee_status yee_step(yee_ctx* c, int64_t n_steps, void* stream) {
  if (!c) return fail(YEE_EINVAL, "NULL context");
  if (!c->bound) return fail(YEE_ESTATE, "no workspace bound");
  if (n_steps < 0) return fail(YEE_EINVAL, "n_steps < 0");
  hipStream_t s = (hipStream_t)stream;
  yee_status st = YEE_OK;
  for (int64_t left = n_steps; left > 0;) {
    const int k = (c->tb_ok && left >= 2 && !c->dbg_count) ? 2 : 1;
    // the probe ring holds series_len steps: fold before a launch would
    // overwrite samples not yet in the DFT
    if (c->n + k - c->folded > c->d.series_len && (st = fold_dft(c, s))) return st;
    if (k == 2) {
      if ((st = launch_two_steps(c, s))) return st;
      c->pecur ^= 1;
    } else if ((st = launch_one_step(c, s))) {
      return st;
    }
    c->n += k;
    c->cur ^= 1;
    left -= k;
  }
  return fold_dft(c, s);
}

yee_status yee_steps_done(const yee_ctx* c, int64_t* n) {
  if (!c || !n) return fail(YEE_EINVAL, "NULL argument");
  *n = c->n;
  return YEE_OK;
}

yee_status yee_read_field(yee_ctx* c, int32_t comp, double* host, void* stream) {
  if (!c || !host) return fail(YEE_EINVAL, "NULL argument");
  if (!c->bound) return fail(YEE_ESTATE, "no workspace bound");
  if (comp < 0 || comp > 5) return fail(YEE_EINVAL, "component %d not in 0..5", comp);
  const auto& d = c->d;
  std::vector<unsigned char> buf((size_t)d.nz * d.ny * c->px * c->tsize);
  hipStream_t s = (hipStream_t)stream;
  const int cur = c->cur;
  HIP_TRY(hipMemcpyAsync(buf.data(), c->ws + c->fields[cur].off + comp * c->comp_bytes, buf.size(),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double dec = d.precision == YEE_F16S ? std::ldexp(1.0, -d.fp16_exp[comp]) : 1.0;
  for (size_t k = 0; k < (size_t)d.nz; ++k)
    for (size_t j = 0; j < (size_t)d.ny; ++j)
      for (size_t i = 0; i < (size_t)d.nx; ++i) {
        const size_t src = (k * d.ny + j) * c->px + i;
        double v;
        if (d.precision == YEE_F64) v = reinterpret_cast<const double*>(buf.data())[src];
        else if (d.precision == YEE_F32) v = reinterpret_cast<const float*>(buf.data())[src];
        else v = (double)reinterpret_cast<const _Float16*>(buf.data())[src] * dec;
        host[(k * d.ny + j) * d.nx + i] = v;
      }
  return YEE_OK;
}

yee_status yee_read_series(yee_ctx* c, int64_t first, int64_t count, double* host, void* stream) {
  if (!c || (count > 0 && !host)) return fail(YEE_EINVAL, "NULL argument");
  if (!c->bound) return fail(YEE_ESTATE, "no workspace bound");
  if (count < 0 || first < 1 || first + count - 1 > c->n || first <= c->n - c->d.series_len)
    return fail(YEE_EINVAL, "samples %lld..%lld not in the ring (steps done %lld, ring %d)",
                (long long)first, (long long)(first + count - 1), (long long)c->n, c->d.series_len);
  const size_t np = c->probes.size();
  if (np == 0 || count == 0) return YEE_OK;
  std::vector<double> ring((size_t)c->d.series_len * np);
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(ring.data(), c->ws + c->series.off, ring.size() * sizeof(double),
                         hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int64_t q = 0; q < count; ++q) {
    const int64_t n = first + q;
    const size_t slot = (size_t)((n - 1) % c->d.series_len);
    std::memcpy(host + q * np, ring.data() + slot * np, np * sizeof(double));
  }
  return YEE_OK;
}

yee_status yee_read_dft(yee_ctx* c, double* re, double* im, void* stream) {
  if (!c || !re || !im) return fail(YEE_EINVAL, "NULL argument");
  if (!c->bound) return fail(YEE_ESTATE, "no workspace bound");
  const size_t cnt = c->probes.size() * c->freqs.size();
  if (cnt == 0) return YEE_OK;
  std::vector<double> buf(2 * cnt);
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemcpyAsync(buf.data(), c->ws + c->dft.off, buf.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (size_t q = 0; q < cnt; ++q) {
    re[q] = buf[2 * q];
    im[q] = buf[2 * q + 1];
  }
  return YEE_OK;
}

static_assert(YEE_FLAG_NONFINITE == yee::kFlagNonFinite && YEE_FLAG_OVERFLOW == yee::kFlagOverflow,
              "status flag bits of the ABI and the kernels differ");

yee_status yee_status_flags(yee_ctx* c, uint32_t* flags, void* stream) {
  if (!c || !flags) return fail(YEE_EINVAL, "NULL argument");
  if (!c->bound) return fail(YEE_ESTATE, "no workspace bound");
  hipStream_t s = (hipStream_t)stream;
  // folding checks the probe samples not yet in the DFT
  yee_status st = fold_dft(c, s);
  if (st) return st;
  const int kind = c->d.precision == YEE_F64 ? 0 : c->d.precision == YEE_F32 ? 1 : 2;
  const size_t nfld = 6 * c->comp_bytes / 16;
  // the probe ring and the DFT accumulators (256-byte aligned, the gap zero)
  const size_t ndbl = (c->dft.off + c->dft.bytes - c->series.off) / 16;
  const size_t words = std::max(nfld, ndbl);
  const int blocks = (int)std::min<size_t>(2048, std::max<size_t>(1, (words + 255) / 256));
  uint32_t* dflags = reinterpret_cast<uint32_t*>(c->ws + c->stat.off);
  hipLaunchKernelGGL(yee::status_scan_kernel, dim3(blocks), dim3(256), 0, s,
                     reinterpret_cast<const uint4*>(c->ws + c->fields[c->cur].off), nfld, kind,
                     reinterpret_cast<const uint4*>(c->ws + c->series.off), ndbl, dflags);
  HIP_TRY(hipGetLastError());
  uint32_t f = 0;
  HIP_TRY(hipMemcpyAsync(&f, dflags, sizeof f, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  *flags = f;
  if (f & YEE_FLAG_OVERFLOW)
    return fail(YEE_EOVERFLOW, "a field sample overflowed FP16 storage by step %lld", (long long)c->n);
  if (f & YEE_FLAG_NONFINITE) return fail(YEE_ENUMERIC, "a non-finite value by step %lld", (long long)c->n);
  return YEE_OK;
}


yee_status yee_state_bytes(const yee_ctx* c, int64_t* bytes) {
  if (!c || !bytes) return fail(YEE_EINVAL, "NULL argument");
  if (!c->bound) return fail(YEE_ESTATE, "no workspace bound");
  *bytes = (int64_t)state_layout(c).total;
  return YEE_OK;
}

yee_status yee_save_state(yee_ctx* c, void* dst, int64_t bytes, void* stream) {
  if (!c || !dst) return fail(YEE_EINVAL, "NULL argument");
  if (!c->bound) return fail(YEE_ESTATE, "no workspace bound");
  const StateLayout L = state_layout(c);
  if (bytes < (int64_t)L.total) return fail(YEE_ENOMEM, "state needs %zu bytes, got %lld", L.total, (long long)bytes);
  hipStream_t s = (hipStream_t)stream;
  unsigned char* o = static_cast<unsigned char*>(dst);
  yee::StateHeader h{};
  state_words(c, h.w);
  hipLaunchKernelGGL(yee::state_header_kernel, dim3(1), dim3(64), 0, s, h, reinterpret_cast<int64_t*>(o));
  HIP_TRY(hipGetLastError());
  const struct { size_t to; const Region& from; size_t n; } parts[] = {
      {L.fields, c->fields[c->cur], 6 * c->comp_bytes}, {L.pse, c->psi_e[c->pecur], c->psi_e[0].bytes},
      {L.psh, c->psi_h[c->cur], c->psi_h[0].bytes},      {L.series, c->series, c->series.bytes},
      {L.dft, c->dft, c->dft.bytes},                     {L.stat, c->stat, c->stat.bytes}};
  for (const auto& p : parts)
    if (p.n) HIP_TRY(hipMemcpyAsync(o + p.to, c->ws + p.from.off, p.n, hipMemcpyDeviceToDevice, s));
  return YEE_OK;
}

yee_status yee_load_state(yee_ctx* c, const void* src, int64_t bytes, void* stream) {
  if (!c || !src) return fail(YEE_EINVAL, "NULL argument");
  if (!c->bound) return fail(YEE_ESTATE, "no workspace bound");
  if (c->in_batch) return fail(YEE_ESTATE, "context is admitted to a batch");
  const StateLayout L = state_layout(c);
  if (bytes < (int64_t)L.total) return fail(YEE_ENOMEM, "state needs %zu bytes, got %lld", L.total, (long long)bytes);
  hipStream_t s = (hipStream_t)stream;
  const unsigned char* in = static_cast<const unsigned char*>(src);
  int64_t got[kStateWords], want[kStateWords];
  HIP_TRY(hipMemcpyAsync(got, in, sizeof got, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  state_words(c, want);
  if (got[0] != kStateMagic) return fail(YEE_EINVAL, "not a saved state (bad magic)");
  for (int q = 1; q < kStateShapeWords; ++q)
    if (got[q] != want[q])
      return fail(YEE_EINVAL, "state was saved from a context of another shape (header word %d: %lld, here %lld)", q,
                  (long long)got[q], (long long)want[q]);
  const int64_t n = got[24], folded = got[25];
  if (n < 0 || folded < 0 || folded > n || n - folded > c->d.series_len)
    return fail(YEE_EINVAL, "corrupt state header (steps %lld, folded %lld)", (long long)n, (long long)folded);
  const struct { Region& to; size_t from; size_t n; } parts[] = {
      {c->fields[0], L.fields, 6 * c->comp_bytes}, {c->psi_e[0], L.pse, c->psi_e[0].bytes},
      {c->psi_h[0], L.psh, c->psi_h[0].bytes},      {c->series, L.series, c->series.bytes},
      {c->dft, L.dft, c->dft.bytes},                {c->stat, L.stat, c->stat.bytes}};
  for (const auto& p : parts)
    if (p.n) HIP_TRY(hipMemcpyAsync(c->ws + p.to.off, in + p.from, p.n, hipMemcpyDeviceToDevice, s));
  c->cur = 0;
  c->pecur = 0;
  c->n = n;
  c->folded = folded;
  return YEE_OK;
}

yee_status yee_sparams(int32_t n_probes, int32_t n_freq, const double* dft_ref_re, const double* dft_ref_im,
                       const double* dft_dut_re, const double* dft_dut_im, int32_t n_ports,
                       const int32_t* port_off, const int32_t* port_probe, const double* port_weight,
                       double* v_ref_re, double* v_ref_im, double* v_dut_re, double* v_dut_im, double* s_re,
                       double* s_im) {
  if (n_probes <= 0 || n_freq <= 0 || n_ports <= 0) return fail(YEE_EINVAL, "sizes must be positive");
  if (!dft_ref_re || !dft_ref_im || !dft_dut_re || !dft_dut_im || !port_off || !port_probe || !port_weight ||
      !s_re || !s_im)
    return fail(YEE_EINVAL, "NULL argument");
  if (port_off[0] != 0) return fail(YEE_EINVAL, "port_off[0] must be 0");
  for (int32_t q = 0; q < n_ports; ++q) {
    if (port_off[q + 1] <= port_off[q]) return fail(YEE_EINVAL, "every port needs at least one probe");
    for (int32_t i = port_off[q]; i < port_off[q + 1]; ++i)
      if (port_probe[i] < 0 || port_probe[i] >= n_probes) return fail(YEE_EINVAL, "port probe index out of range");
  }
  using cd = std::complex<double>;
  for (int32_t q = 0; q < n_ports; ++q) {
    for (int32_t f = 0; f < n_freq; ++f) {
      cd vr = 0.0, vd = 0.0;
      for (int32_t i = port_off[q]; i < port_off[q + 1]; ++i) {
        const size_t x = (size_t)port_probe[i] * n_freq + f;
        vr += port_weight[i] * cd(dft_ref_re[x], dft_ref_im[x]);
        vd += port_weight[i] * cd(dft_dut_re[x], dft_dut_im[x]);
      }
      const size_t o = (size_t)q * n_freq + f;
      if (v_ref_re) v_ref_re[o] = vr.real();
      if (v_ref_im) v_ref_im[o] = vr.imag();
      if (v_dut_re) v_dut_re[o] = vd.real();
      if (v_dut_im) v_dut_im[o] = vd.imag();
      const cd sq = (q == 0 ? vd - vr : vd) / vr;
      s_re[o] = sq.real();
      s_im[o] = sq.imag();
    }
  }
  return YEE_OK;
}

// ---------------------------------------------------------------------------
// Batched stepper (continuous batching of many grids)
// ---------------------------------------------------------------------------
yee_status yee_batch_footprint(int32_t max_slots, int64_t* bytes) {
  if (max_slots < 1 || !bytes) return fail(YEE_EINVAL, "max_slots must be >= 1");
  *bytes = (int64_t)(256 + align256((size_t)max_slots * batch_desc_bytes()));
  return YEE_OK;
}

yee_status yee_batch_create(int32_t max_slots, int64_t hbm_budget, int32_t steps_per_replay, yee_batch** out) {
  if (!out) return fail(YEE_EINVAL, "out is NULL");
  *out = nullptr;
  if (max_slots < 1 || max_slots > 4096 || hbm_budget <= 0 || steps_per_replay < 1 || steps_per_replay > 4096)
    return fail(YEE_EINVAL, "bad batch parameters (slots %d, budget %lld, steps per replay %d)", max_slots,
                (long long)hbm_budget, steps_per_replay);
  auto* b = new (std::nothrow) yee_batch();
  if (!b) return fail(YEE_ENOMEM, "host allocation failed");
  b->max_slots = max_slots;
  b->budget = hbm_budget;
  b->K = steps_per_replay;
  b->slots.resize(max_slots);
  b->lds = batch_lds_bytes(b->prec);
  *out = b;
  return YEE_OK;
}

yee_status yee_batch_set_precision(yee_batch* b, int32_t precision) {
  if (!b) return fail(YEE_EINVAL, "NULL batch");
  if (precision != YEE_F64 && precision != YEE_F32 && precision != YEE_F16S)
    return fail(YEE_EINVAL, "unknown precision %d", precision);
  if (b->bound) return fail(YEE_ESTATE, "the precision is set before yee_batch_bind_workspace");
  b->prec = precision;
  b->lds = batch_lds_bytes(precision);
  return YEE_OK;
}

void yee_batch_destroy(yee_batch* b) {
  if (!b) return;
  for (auto& sl : b->slots)
    if (sl.used && sl.ctx) sl.ctx->in_batch = false;
  for (int i = 0; i < 2; ++i) {
    if (b->staged[i]) {
      (void)hipEventSynchronize(b->staged[i]);
      (void)hipEventDestroy(b->staged[i]);
    }
    if (b->staging[i]) (void)hipHostFree(b->staging[i]);
  }
  for (int i = 0; i < 2; ++i) {
    if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
    if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
  }
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
}

yee_status yee_batch_bind_workspace(yee_batch* b, void* dev, int64_t bytes) {
  if (!b || !dev) return fail(YEE_EINVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(dev) & 255) return fail(YEE_EINVAL, "workspace must be 256-byte aligned");
  int64_t need = 0;
  yee_batch_footprint(b->max_slots, &need);
  if (bytes < need) return fail(YEE_ENOMEM, "batch workspace has %lld bytes, needs %lld", (long long)bytes, (long long)need);
  int dev_id = 0, cus = 0, per_cu = 0;
  HIP_TRY(hipGetDevice(&dev_id));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev_id));
  // the persistent launch: as many workgroups as are resident at once
  const int bt = yee::kWave * kBatchBlockWaves;
  if (b->prec == YEE_F16S)
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, yee::batch_step_kernel<_Float16, float, 2>, bt, b->lds));
  else if (b->prec == YEE_F64)
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, yee::batch_step_kernel<double, double, 1>, bt, b->lds));
  else
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, yee::batch_step_kernel<float, float, 1>, bt, b->lds));
  b->grid = std::max(8, std::max(1, per_cu) * cus);
  b->staging_bytes = 256 + (size_t)b->max_slots * batch_desc_bytes();
  for (int i = 0; i < 2; ++i) {
    if (!b->staging[i]) HIP_TRY(hipHostMalloc(reinterpret_cast<void**>(&b->staging[i]), b->staging_bytes, 0));
    if (!b->staged[i]) HIP_TRY(hipEventCreateWithFlags(&b->staged[i], hipEventDisableTiming));
  }
  b->ws = static_cast<unsigned char*>(dev);
  b->ws_bytes = bytes;
  b->bound = true;
  return YEE_OK;
}

namespace {
// (y-tile, plane) units of the unfinished slots, and their tiles at kz planes per chunk
int64_t batch_units(const yee_batch* b) {
  int64_t u = 0;
  for (auto& sl : b->slots)
    if (sl.used && sl.ctx->n < sl.n_end) u += (int64_t)((sl.ctx->d.ny + sl.ty - 1) / sl.ty) * sl.ctx->d.nz;
  return u;
}
int64_t batch_tiles(const yee_batch* b, int kz) {
  int64_t t = 0;
  for (auto& sl : b->slots)
    if (sl.used && sl.ctx->n < sl.n_end)
      t += (int64_t)((sl.ctx->d.ny + sl.ty - 1) / sl.ty) * ((sl.ctx->d.nz + kz - 1) / kz);
  return t;
}
}  // namespace

yee_status yee_batch_admit(yee_batch* b, yee_ctx* c, int64_t n_steps, int32_t* slot) {
  if (!b || !c || !slot) return fail(YEE_EINVAL, "NULL argument");
  if (!b->bound) return fail(YEE_ESTATE, "batch workspace not bound");
  if (!c->bound) return fail(YEE_ESTATE, "context workspace not bound");
  if (n_steps < 1) return fail(YEE_EINVAL, "n_steps must be >= 1");
  if (c->d.precision != b->prec)
    return fail(YEE_EINVAL, "the batch runs contexts of precision %d (yee_batch_set_precision), this one is %d", b->prec,
                (int)c->d.precision);
  const int bV = batch_V(b->prec);
  if (c->d.nx > 4 * yee::kWave * bV)
    return fail(YEE_EINVAL, "the batched stepper takes rows of at most %d samples", 4 * yee::kWave * bV);
  if (!c->probes.empty() && c->d.series_len < b->K)
    return fail(YEE_EINVAL, "probe ring (%d) shorter than the steps per replay (%d)", c->d.series_len, b->K);
  for (auto& sl : b->slots)
    if (sl.used && sl.ctx == c) return fail(YEE_EINVAL, "context already admitted");
  if (b->in_use + c->ws_bytes > b->budget) return fail(YEE_EAGAIN, "HBM budget exhausted");
  for (int32_t q = 0; q < b->max_slots; ++q) {
    auto& sl = b->slots[q];
    if (sl.used) continue;
    sl.used = true;
    sl.ctx = c;
    sl.n_end = c->n + n_steps;
    sl.bytes = c->ws_bytes;
    sl.ty = batch_tile_rows(c, bV);
    c->in_batch = true;
    b->in_use += sl.bytes;
    *slot = q;
    return YEE_OK;
  }
  return fail(YEE_EAGAIN, "no free slot");
}

}  // extern "C"

namespace {

// One replay of a batch whose contexts store T and compute in C, V samples
// per lane (see yee_batch_run).
template <class T, class C, int V>
yee_status batch_run_t(yee_batch* b, hipStream_t s) {
  using BatchDesc = yee::SlotDesc<T, C>;
  // The device table is rewritten by a copy on `stream`, behind the replays
  // already queued there, so the host runs ahead of the device; only the host
  // image used two runs ago must have been copied out.
  const int sb = (int)(b->runs & 1);
  if (b->staged_used[sb]) HIP_TRY(hipEventSynchronize(b->staged[sb]));
  const size_t hdr_bytes = 256;
  unsigned char* stg = b->staging[sb];
  std::memset(stg, 0, b->staging_bytes);
  BatchDesc* desc = reinterpret_cast<BatchDesc*>(stg + hdr_bytes);
  int32_t nact = 0, tiles = 0;
  size_t comp_total = 0;
  std::vector<int32_t> order;
  // planes per chunk for this replay: the fewest (kBatchMinChunk ..
  // kBatchMaxChunk) that spread the (y-tile, plane) units of every active slot
  // over the resident workgroups in one round -- short marches when few
  // requests run, long ones (less warm-up) when many do
  int kz_all = (int)std::min<int64_t>(kBatchMaxChunk,
                                      std::max<int64_t>(kBatchMinChunk, (batch_units(b) + b->grid - 1) / b->grid));
  while (kz_all < kBatchMaxChunk && batch_tiles(b, kz_all) > b->grid) ++kz_all;
  for (int32_t q = 0; q < b->max_slots; ++q) {
    auto& sl = b->slots[q];
    if (!sl.used || sl.ctx->n >= sl.n_end) continue;
    yee_ctx* c = sl.ctx;
    BatchDesc& d = desc[nact++];
    sl.kz = std::min(c->d.nz, kz_all);
    d.a = fill_args<T, C>(c, V, sl.ty, sl.kz);
    // set[0] holds the state at the start of the replay (the context's current buffers)
    d.set[0] = reinterpret_cast<const T*>(c->ws + c->fields[c->cur].off);
    d.set[1] = reinterpret_cast<const T*>(c->ws + c->fields[c->cur ^ 1].off);
    d.psh[0] = reinterpret_cast<C*>(c->ws + c->psi_h[c->cur].off);
    d.psh[1] = reinterpret_cast<C*>(c->ws + c->psi_h[c->cur ^ 1].off);
    d.base_n = c->n;
    d.n_end = sl.n_end;
    d.series_len = c->d.series_len;
    d.tile0 = tiles;
    tiles += d.a.ntiles;
    comp_total += c->comp_bytes;
    order.push_back(q);
  }
  if (nact == 0) return YEE_OK;
  reinterpret_cast<int32_t*>(stg)[0] = nact;
  reinterpret_cast<int32_t*>(stg)[1] = tiles;
  HIP_TRY(hipMemcpyAsync(b->ws, stg, hdr_bytes + (size_t)nact * sizeof(BatchDesc), hipMemcpyHostToDevice, s));
  HIP_TRY(hipEventRecord(b->staged[sb], s));
  b->staged_used[sb] = true;
  b->runs += 1;
  // the replay steps every active slot: their fields share the cache
  const int nt = stream_stores(comp_total) ? 1 : 0;
  if (!b->exec[nt]) {
    // capture K launches once per store policy; they read the descriptor
    // table from device memory
    const BatchDesc* dslots = reinterpret_cast<const BatchDesc*>(b->ws + hdr_bytes);
    const int32_t* dhdr = reinterpret_cast<const int32_t*>(b->ws);
    // (captured on a private stream: the caller's may be the legacy null stream)
    if (!b->capture) HIP_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
    HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
    const dim3 block(yee::kWave * kBatchBlockWaves);
    for (int q = 0; q < b->K; ++q) {
      if (nt)
        hipLaunchKernelGGL((yee::batch_step_kernel<T, C, V, yee::kStream>), dim3(b->grid), block, b->lds, b->capture,
                           dslots, dhdr, q);
      else
        hipLaunchKernelGGL((yee::batch_step_kernel<T, C, V>), dim3(b->grid), block, b->lds, b->capture, dslots, dhdr,
                           q);
    }
    hipGraph_t g = nullptr;
    hipError_t e1 = hipStreamEndCapture(b->capture, &g);
    if (e1 != hipSuccess) return fail(YEE_EHIP, "graph capture failed: %s", hipGetErrorString(e1));
    b->graph[nt] = g;
    HIP_TRY(hipGraphInstantiate(&b->exec[nt], b->graph[nt], nullptr, nullptr, 0));
  }
  HIP_TRY(hipGraphLaunch(b->exec[nt], s));
  // host bookkeeping: every included slot advanced min(K, remaining) steps
  for (int32_t q : order) {
    auto& sl = b->slots[q];
    yee_ctx* c = sl.ctx;
    const int64_t taken = std::min(sl.n_end, c->n + b->K) - c->n;
    c->n += taken;
    c->cur ^= (int)(taken & 1);
    yee_status st = fold_dft(c, s);
    if (st) return st;
  }
  return YEE_OK;
}

}  // namespace

extern "C" {

yee_status yee_batch_run(yee_batch* b, void* stream) {
  if (!b) return fail(YEE_EINVAL, "NULL batch");
  if (!b->bound) return fail(YEE_ESTATE, "batch workspace not bound");
  hipStream_t s = (hipStream_t)stream;
  if (b->prec == YEE_F16S) return batch_run_t<_Float16, float, 2>(b, s);
  if (b->prec == YEE_F64) return batch_run_t<double, double, 1>(b, s);
  return batch_run_t<float, float, 1>(b, s);
}

yee_status yee_batch_poll(yee_batch* b, int32_t* done, int32_t cap, int32_t* n_done) {
  if (!b || !n_done || (cap > 0 && !done)) return fail(YEE_EINVAL, "NULL argument");
  int32_t m = 0;
  for (int32_t q = 0; q < b->max_slots; ++q) {
    const auto& sl = b->slots[q];
    if (sl.used && sl.ctx->n >= sl.n_end) {
      if (m < cap) done[m] = q;
      ++m;
    }
  }
  *n_done = m;
  return YEE_OK;
}

yee_status yee_batch_release(yee_batch* b, int32_t slot) {
  if (!b || slot < 0 || slot >= b->max_slots) return fail(YEE_EINVAL, "bad slot");
  auto& sl = b->slots[slot];
  if (!sl.used) return fail(YEE_ESTATE, "slot %d is free", slot);
  b->in_use -= sl.bytes;
  sl.ctx->in_batch = false;
  sl = yee_batch::Slot{};
  return YEE_OK;
}

yee_status yee_batch_info(const yee_batch* b, int32_t* active, int64_t* bytes_in_use) {
  if (!b || !active || !bytes_in_use) return fail(YEE_EINVAL, "NULL argument");
  int32_t a = 0;
  for (const auto& sl : b->slots) a += sl.used ? 1 : 0;
  *active = a;
  *bytes_in_use = b->in_use;
  return YEE_OK;
}

}  // extern "C"

// ===========================================================================
// Discrete adjoint (reverse-mode derivative of J = sum_n sum_p y_p[n]^2 with
// respect to eps_r of the cells of a box), with checkpoint-recompute.
// ===========================================================================
struct yee_adjoint {
  yee_ctx* c = nullptr;
  int64_t N = 0;          // steps of the forward run
  int32_t K = 0;          // steps between checkpoints
  int32_t S = 0;          // segments: ceil(N / K)
  int32_t box[6] = {};    // i0, i1, j0, j1, k0, k1
  int32_t bx = 0, by = 0, bz = 0;
  size_t nbox = 0;
  bool bound = false;
  unsigned char* ws = nullptr;
  int64_t ws_bytes = 0;
  Region ckpt, hist, u, hb, pe[2], ph[2], phist, jout, dcoef, inj;
  size_t ckpt_bytes = 0;  // one checkpoint: fields | psi_E | psi_H
  size_t ucomp = 0;       // bytes of one adjoint component array
  int32_t H = 1;          // history slots: segments whose E history is kept
  std::vector<int32_t> slot_seg;  // segment held by each history slot (-1: none)
  bool have_forward = false;
  std::vector<yee::InjDev> inj_host;
  std::vector<double> dcoef_host;
};

namespace {

void adj_layout(yee_adjoint* A) {
  const yee_ctx* c = A->c;
  const auto& d = c->d;
  size_t off = 0;
  auto take = [&](Region& r, size_t bytes) {
    r.off = off;
    r.bytes = bytes;
    off += align256(std::max<size_t>(bytes, 1));
  };
  A->ckpt_bytes = align256(6 * c->comp_bytes) + 2 * align256(c->psi_e[0].bytes);
  take(A->ckpt, (size_t)(A->S + 1) * A->ckpt_bytes);
  take(A->hist, (size_t)A->H * (A->K + 1) * 3 * A->nbox * c->tsize);
  A->ucomp = align256((size_t)d.nz * d.ny * c->px * c->csize);
  take(A->u, 3 * A->ucomp);
  take(A->hb, 3 * A->ucomp);
  for (int q = 0; q < 2; ++q) take(A->pe[q], c->psi_e[0].bytes);
  for (int q = 0; q < 2; ++q) take(A->ph[q], c->psi_e[0].bytes);
  take(A->phist, (size_t)A->N * c->probes.size() * sizeof(double));
  take(A->jout, sizeof(double));
  take(A->dcoef, (size_t)c->nsx * c->nsy * c->nsz * 2 * sizeof(double));
  take(A->inj, c->probes.size() * sizeof(yee::InjDev));
  A->ws_bytes = (int64_t)off;
}

yee_status adj_copy(void* dst, const void* src, size_t bytes, hipStream_t s) {
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, s));
  return YEE_OK;
}

// Checkpoint slot q <-> the context's current state (fields, psi_E, psi_H).
yee_status adj_checkpoint(yee_adjoint* A, int q, bool save, hipStream_t s) {
  yee_ctx* c = A->c;
  const int cur = c->cur;
  unsigned char* slot = A->ws + A->ckpt.off + (size_t)q * A->ckpt_bytes;
  unsigned char* parts[3] = {slot, slot + align256(6 * c->comp_bytes),
                             slot + align256(6 * c->comp_bytes) + align256(c->psi_e[0].bytes)};
  unsigned char* live[3] = {c->ws + c->fields[cur].off, c->ws + c->psi_e[c->pecur].off, c->ws + c->psi_h[cur].off};
  const size_t bytes[3] = {6 * c->comp_bytes, c->psi_e[0].bytes, c->psi_e[0].bytes};
  for (int p = 0; p < 3; ++p) {
    yee_status st = save ? adj_copy(parts[p], live[p], bytes[p], s) : adj_copy(live[p], parts[p], bytes[p], s);
    if (st) return st;
  }
  return YEE_OK;
}

// Destination of entry m of history slot `slot` (component 0; components hs apart).
void* adj_hist_entry(yee_adjoint* A, int slot, int m) {
  const size_t hs = A->nbox;
  return A->ws + A->hist.off + ((size_t)slot * (A->K + 1) + m) * 3 * hs * A->c->csize;
}

// One forward step of the context that also writes E^{n+1} of the box into
// entry m of history slot `slot` (no separate copy kernel).
yee_status adj_step_store(yee_adjoint* A, int slot, int m, bool record, hipStream_t s) {
  const HistOut h{A->box, adj_hist_entry(A, slot, m), (uint64_t)A->nbox};
  return launch_one_step(A->c, s, record, &h);
}

// E of the box cells at the current step into entry m of history slot `slot`.
yee_status adj_store(yee_adjoint* A, int slot, int m, hipStream_t s) {
  yee_ctx* c = A->c;
  const int cur = c->cur;
  const int4 lo = {A->box[0], A->box[2], A->box[4], 0};
  const dim3 grid((A->bx + yee::kAdjBX - 1) / yee::kAdjBX, (A->by + yee::kAdjBY - 1) / yee::kAdjBY, A->bz);
  const dim3 block(yee::kAdjBX, yee::kAdjBY);
  const uint64_t hs = A->nbox;
  if (c->d.precision == YEE_F64) {
    const double* f = reinterpret_cast<const double*>(c->ws + c->fields[cur].off);
    double* dst = reinterpret_cast<double*>(A->ws + A->hist.off) + ((size_t)slot * (A->K + 1) + m) * 3 * hs;
    hipLaunchKernelGGL(yee::adj_store_kernel<double>, grid, block, 0, s, f, (uint64_t)(c->comp_bytes / 8),
                       c->d.ny, c->px, lo, A->bx, A->by, dst, hs);
  } else {
    const float* f = reinterpret_cast<const float*>(c->ws + c->fields[cur].off);
    float* dst = reinterpret_cast<float*>(A->ws + A->hist.off) + ((size_t)slot * (A->K + 1) + m) * 3 * hs;
    hipLaunchKernelGGL(yee::adj_store_kernel<float>, grid, block, 0, s, f, (uint64_t)(c->comp_bytes / 4),
                       c->d.ny, c->px, lo, A->bx, A->by, dst, hs);
  }
  HIP_TRY(hipGetLastError());
  return YEE_OK;
}

// Probe samples of steps s0+1 .. s0+count from the ring into the full history.
yee_status adj_gather(yee_adjoint* A, int64_t s0, int64_t count, hipStream_t s) {
  yee_ctx* c = A->c;
  const int np = (int)c->probes.size();
  if (np == 0 || count <= 0) return YEE_OK;
  const int total = (int)(count * np);
  hipLaunchKernelGGL(yee::adj_gather_kernel, dim3((total + 255) / 256), dim3(256), 0, s,
                     reinterpret_cast<const double*>(c->ws + c->series.off), np, c->d.series_len, s0, (int)count,
                     reinterpret_cast<double*>(A->ws + A->phist.off));
  HIP_TRY(hipGetLastError());
  return YEE_OK;
}

template <class T, class C>
yee::AdjArgs<T, C> adj_args(yee_adjoint* A, int64_t n, int slot, int m, int pin, int pout, bool e_side) {
  using namespace yee;
  yee_ctx* c = A->c;
  const auto& d = c->d;
  AdjArgs<T, C> a{};
  a.u = reinterpret_cast<C*>(A->ws + A->u.off);
  a.hb = reinterpret_cast<C*>(A->ws + A->hb.off);
  a.ustride = A->ucomp / sizeof(C);
  const Region* pr = e_side ? A->ph : A->pe;
  a.pin = reinterpret_cast<const C*>(A->ws + pr[pin].off);
  a.pout = reinterpret_cast<C*>(A->ws + pr[pout].off);
  for (int q = 0; q < 6; ++q) a.psoff[q] = c->psi_off[q];
  a.prof = reinterpret_cast<const C*>(c->ws + c->prof.off);
  a.plen = (int32_t)c->prof_len;
  a.seg = reinterpret_cast<const int32_t*>(c->ws + c->segr.off);
  a.coef = reinterpret_cast<const Coef2<C>*>(c->ws + c->coef.off);
  a.dcoef = reinterpret_cast<const double2*>(A->ws + A->dcoef.off);
  a.nsx = c->nsx;
  a.nsxy = c->nsx * c->nsy;
  a.pec_plane = reinterpret_cast<const int32_t*>(c->ws + c->pecplane.off);
  a.pec_mask = reinterpret_cast<const uint8_t*>(c->ws + c->pecmask.off);
  const T* h0 = reinterpret_cast<const T*>(A->ws + A->hist.off) + (size_t)slot * (A->K + 1) * 3 * A->nbox;
  a.hstride = A->nbox;
  a.hist_n = h0 + (size_t)m * 3 * A->nbox;
  a.hist_np1 = h0 + (size_t)(m + 1) * 3 * A->nbox;
  for (int q = 0; q < 6; ++q) a.box[q] = A->box[q];
  a.src = reinterpret_cast<const SrcDev*>(c->ws + c->srcr.off);
  a.nsrc = (int32_t)c->src.size();
  a.n = n;
  a.dt = c->dt;
  a.nx = d.nx; a.ny = d.ny; a.nz = d.nz; a.px = c->px;
  for (int q = 0; q < 3; ++q) a.L[q] = d.cpml_cells[q];
  a.inv_d[0] = static_cast<C>(1.0 / d.dx);
  a.inv_d[1] = static_cast<C>(1.0 / d.dy);
  a.inv_d[2] = static_cast<C>(1.0 / d.dz);
  a.dt_mu = static_cast<C>(c->dt / kMu0);
  a.inj = reinterpret_cast<const InjDev*>(A->ws + A->inj.off);
  a.ninj = (int32_t)A->inj_host.size();
  a.probe = reinterpret_cast<const int4*>(c->ws + c->prober.off);
  a.nprobe = (int32_t)c->probes.size();
  a.rowflag = reinterpret_cast<const uint8_t*>(c->ws + c->rowflag.off);
  a.yrow_h = nullptr;
  a.yrow_e = nullptr;
  return a;
}

// One reverse step of forward step n (n0 <= n < n0 + K: entry m = n - n0 of
// history slot `slot`).
template <class C>
yee_status adj_reverse_step(yee_adjoint* A, int64_t n, int slot, int m, int& pe, int& ph, double* grad,
                            hipStream_t s) {
  using namespace yee;
  yee_ctx* c = A->c;
  const auto& d = c->d;
  const int np = (int)c->probes.size();
  const int ninj = (int)A->inj_host.size();
  const double* yrow = reinterpret_cast<const double*>(A->ws + A->phist.off);
  // The objective seeds of step n: the E ones were added by the previous
  // reverse step's adj_e, except before the first reverse step; the H ones
  // are added by adj_h below.
  if (ninj > 0 && n == A->N - 1) {
    hipLaunchKernelGGL(adj_inject_kernel<C>, dim3((ninj + 63) / 64), dim3(64), 0, s,
                       reinterpret_cast<const InjDev*>(A->ws + A->inj.off), ninj,
                       reinterpret_cast<const int4*>(c->ws + c->prober.off), np, yrow + (size_t)n * np,
                       reinterpret_cast<C*>(A->ws + A->u.off), reinterpret_cast<C*>(A->ws + A->hb.off),
                       (uint64_t)(A->ucomp / sizeof(C)), 3);
    HIP_TRY(hipGetLastError());
  }
  const dim3 grid((d.nx + kAdjBX - 1) / kAdjBX, (d.ny + kAdjBY - 1) / kAdjBY, d.nz);
  const dim3 block(kAdjBX, kAdjBY);
  AdjArgs<C, C> ah = adj_args<C, C>(A, n, slot, m, pe, pe ^ 1, false);
  ah.yrow_h = ninj > 0 ? yrow + (size_t)n * np : nullptr;
  hipLaunchKernelGGL(adj_h_kernel<C>, grid, block, 0, s, ah);
  HIP_TRY(hipGetLastError());
  pe ^= 1;
  AdjArgs<C, C> ae = adj_args<C, C>(A, n, slot, m, ph, ph ^ 1, true);
  ae.yrow_e = (ninj > 0 && n > 0) ? yrow + (size_t)(n - 1) * np : nullptr;
  ae.grad = grad;
  hipLaunchKernelGGL((adj_e_kernel<C, C>), grid, block, 0, s, ae);
  HIP_TRY(hipGetLastError());
  ph ^= 1;
  return YEE_OK;
}

}  // namespace

extern "C" {

yee_status yee_adjoint_create(yee_ctx* c, int64_t n_steps, int32_t checkpoint_every, const int32_t* box,
                              yee_adjoint** out) {
  if (!out) return fail(YEE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!c || !box) return fail(YEE_EINVAL, "NULL argument");
  if (!c->bound) return fail(YEE_ESTATE, "context workspace not bound");
  if (c->d.precision == YEE_F16S) return fail(YEE_EINVAL, "the adjoint runs FP64 or FP32 contexts");
  if (n_steps < 1 || checkpoint_every < 1) return fail(YEE_EINVAL, "n_steps and checkpoint_every must be >= 1");
  const int n3[3] = {c->d.nx, c->d.ny, c->d.nz};
  for (int q = 0; q < 3; ++q)
    if (box[2 * q] < 0 || box[2 * q] >= box[2 * q + 1] || box[2 * q + 1] > n3[q])
      return fail(YEE_EINVAL, "box [%d, %d) invalid on an axis of %d cells", box[2 * q], box[2 * q + 1], n3[q]);
  if (c->d.nz > 65535) return fail(YEE_EINVAL, "the adjoint kernels take nz <= 65535");
  const int64_t S = (n_steps + checkpoint_every - 1) / checkpoint_every;
  if (S > (1 << 20)) return fail(YEE_EINVAL, "too many checkpoints (%lld)", (long long)S);
  if ((uint64_t)n_steps * c->probes.size() >= (1ull << 31))
    return fail(YEE_EINVAL, "probe history of %lld steps too long", (long long)n_steps);
  auto* A = new (std::nothrow) yee_adjoint();
  if (!A) return fail(YEE_ENOMEM, "host allocation failed");
  A->c = c;
  A->N = n_steps;
  A->K = (int32_t)std::min<int64_t>(checkpoint_every, n_steps);
  A->S = (int32_t)S;
  for (int q = 0; q < 6; ++q) A->box[q] = box[q];
  A->bx = box[1] - box[0];
  A->by = box[3] - box[2];
  A->bz = box[5] - box[4];
  A->nbox = (size_t)A->bx * A->by * A->bz;
  A->slot_seg.assign(1, -1);
  adj_layout(A);
  *out = A;
  return YEE_OK;
}

yee_status yee_adjoint_set_history(yee_adjoint* A, int32_t segments) {
  if (!A) return fail(YEE_EINVAL, "NULL argument");
  if (A->bound) return fail(YEE_ESTATE, "set the history before binding the workspace");
  if (segments < 0 || segments > A->S)
    return fail(YEE_EINVAL, "history of %d segments: must be 0 (all) to %d", segments, A->S);
  A->H = segments == 0 ? A->S : segments;
  A->slot_seg.assign((size_t)A->H, -1);
  adj_layout(A);
  return YEE_OK;
}

void yee_adjoint_destroy(yee_adjoint* A) { delete A; }

yee_status yee_adjoint_footprint(const yee_adjoint* A, int64_t* bytes) {
  if (!A || !bytes) return fail(YEE_EINVAL, "NULL argument");
  *bytes = A->ws_bytes;
  return YEE_OK;
}

yee_status yee_adjoint_bind_workspace(yee_adjoint* A, void* dev, int64_t bytes) {
  if (!A || !dev) return fail(YEE_EINVAL, "NULL argument");
  if (reinterpret_cast<uintptr_t>(dev) & 255) return fail(YEE_EINVAL, "workspace must be 256-byte aligned");
  if (bytes < A->ws_bytes)
    return fail(YEE_ENOMEM, "adjoint workspace has %lld bytes, needs %lld", (long long)bytes, (long long)A->ws_bytes);
  A->ws = static_cast<unsigned char*>(dev);
  A->bound = true;
  A->have_forward = false;
  A->slot_seg.assign((size_t)A->H, -1);
  return YEE_OK;
}

yee_status yee_adjoint_forward(yee_adjoint* A, double* objective, void* stream) {
  if (!A || !objective) return fail(YEE_EINVAL, "NULL argument");
  if (!A->bound) return fail(YEE_ESTATE, "adjoint workspace not bound");
  yee_ctx* c = A->c;
  if (c->n != 0) return fail(YEE_ESTATE, "the forward run starts at step 0 (context is at step %lld)", (long long)c->n);
  hipStream_t s = (hipStream_t)stream;
  const auto& d = c->d;
  A->have_forward = false;
  yee_status st = YEE_OK;
  int64_t gathered = 0;
  // the newest H segments keep the E history of the box from this run
  const int32_t kept0 = A->S - A->H;
  A->slot_seg.assign((size_t)A->H, -1);
  for (int32_t seg = 0; seg < A->S; ++seg) {
    const int64_t n0 = (int64_t)seg * A->K, n1 = std::min(A->N, n0 + A->K);
    const bool keep = seg >= kept0;
    const int slot = seg - kept0;
    if ((st = adj_checkpoint(A, seg, true, s))) return st;
    if (keep && (st = adj_store(A, slot, 0, s))) return st;
    for (int64_t n = n0; n < n1; ++n) {
      if ((st = keep ? adj_step_store(A, slot, (int)(n + 1 - n0), true, s) : launch_one_step(c, s))) return st;
      c->n += 1;
      c->cur ^= 1;
      if (c->n - gathered >= d.series_len) {
        if ((st = adj_gather(A, gathered, c->n - gathered, s))) return st;
        gathered = c->n;
      }
      if (c->n - c->folded >= d.series_len && (st = fold_dft(c, s))) return st;
    }
  }
  if ((st = adj_gather(A, gathered, c->n - gathered, s))) return st;
  if ((st = fold_dft(c, s))) return st;
  if ((st = adj_checkpoint(A, A->S, true, s))) return st;
  // Tables only the backward run reads, built on the host while the queued
  // steps run on the device:
  // derivative table per block: (dCa/deps_r / Cb, dCb/deps_r / Cb^2) in FP64
  const size_t nb = (size_t)c->nsx * c->nsy * c->nsz;
  A->dcoef_host.assign(2 * nb, 0.0);
  for (size_t b = 0; b < nb; ++b) {
    const double er = c->eps[b];
    const double sg = c->sig[b] * c->dt / (2.0 * kEps0 * er);
    const double cb = (c->dt / (kEps0 * er)) / (1.0 + sg);
    const double dca = 2.0 * sg / (er * (1.0 + sg) * (1.0 + sg));
    const double dcb = -cb / (er * (1.0 + sg));
    A->dcoef_host[2 * b] = dca / cb;
    A->dcoef_host[2 * b + 1] = dcb / (cb * cb);
  }
  // unique probed samples and their injection weights (2 Cb as the step uses it)
  A->inj_host.clear();
  const int np = (int)c->probes.size();
  for (int p = 0; p < np; ++p) {
    const int4 pr = c->probes[p];
    bool seen = false;
    for (int q = 0; q < p && !seen; ++q) {
      const int4 o = c->probes[q];
      seen = o.x == pr.x && o.y == pr.y && o.z == pr.z && o.w == pr.w;
    }
    if (seen) continue;
    yee::InjDev e{};
    e.comp = pr.x; e.i = pr.y; e.j = pr.z; e.k = pr.w; e.first = p;
    e.off = (uint32_t)(((size_t)pr.w * d.ny + pr.z) * c->px + pr.y);
    e.w = 2.0;
    if (pr.x < 3) {
      const int i = pr.y, j = pr.z, k = pr.w;
      bool upd = pr.x == 0 ? (j > 0 && k > 0) : pr.x == 1 ? (i > 0 && k > 0) : (i > 0 && j > 0);
      for (size_t q = 0; q < c->pec_k.size(); ++q)
        if (c->pec_k[q] == k && (c->pec_masks[q][(size_t)j * c->px + i] >> pr.x & 1)) upd = false;
      const size_t b = (size_t)c->segx[i] + (size_t)c->segy[j] * c->nsx + (size_t)c->segz[k] * c->nsx * c->nsy;
      const double eps = kEps0 * c->eps[b];
      const double sg = c->sig[b] * c->dt / (2.0 * eps);
      const double cb = (c->dt / eps) / (1.0 + sg);
      const double cbc = c->csize == 8 ? cb : (double)(float)cb;
      e.w = upd ? 2.0 * cbc : 0.0;
    }
    A->inj_host.push_back(e);
  }
  HIP_TRY(hipMemcpyAsync(A->ws + A->dcoef.off, A->dcoef_host.data(), A->dcoef_host.size() * sizeof(double),
                         hipMemcpyHostToDevice, s));
  if (!A->inj_host.empty())
    HIP_TRY(hipMemcpyAsync(A->ws + A->inj.off, A->inj_host.data(), A->inj_host.size() * sizeof(yee::InjDev),
                           hipMemcpyHostToDevice, s));

  hipLaunchKernelGGL(yee::adj_objective_kernel, dim3(1), dim3(256), 0, s,
                     reinterpret_cast<const double*>(A->ws + A->phist.off), (int64_t)A->N * np,
                     reinterpret_cast<double*>(A->ws + A->jout.off));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(objective, A->ws + A->jout.off, sizeof(double), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  for (int32_t q = 0; q < A->H; ++q) A->slot_seg[q] = kept0 + q;
  A->have_forward = true;
  return YEE_OK;
}

yee_status yee_adjoint_backward(yee_adjoint* A, double* grad, void* stream) {
  if (!A || !grad) return fail(YEE_EINVAL, "NULL argument");
  if (!A->bound || !A->have_forward) return fail(YEE_ESTATE, "no forward run recorded");
  yee_ctx* c = A->c;
  if (c->n != A->N) return fail(YEE_ESTATE, "context was stepped after the forward run");
  hipStream_t s = (hipStream_t)stream;
  HIP_TRY(hipMemsetAsync(A->ws + A->u.off, 0, A->ph[1].off + A->ph[1].bytes - A->u.off, s));
  HIP_TRY(hipMemsetAsync(grad, 0, A->nbox * sizeof(double), s));
  int pe = 0, ph = 0;
  yee_status st = YEE_OK;
  for (int32_t seg = A->S - 1; seg >= 0; --seg) {
    const int64_t n0 = (int64_t)seg * A->K, n1 = std::min(A->N, n0 + A->K);
    int slot = -1;
    for (int32_t q = 0; q < A->H; ++q)
      if (A->slot_seg[q] == seg) slot = q;
    if (slot < 0) {
      // recompute the segment from its checkpoint into slot 0, whose segment
      // (newer than this one) has been walked already
      slot = 0;
      c->n = n0;
      if ((st = adj_checkpoint(A, seg, false, s))) return st;
      if ((st = adj_store(A, slot, 0, s))) return st;
      for (int64_t n = n0; n < n1; ++n) {
        if ((st = adj_step_store(A, slot, (int)(n + 1 - n0), false, s))) return st;
        c->n += 1;
        c->cur ^= 1;
      }
      A->slot_seg[slot] = seg;
    }
    for (int64_t n = n1 - 1; n >= n0; --n) {
      st = c->csize == 8 ? adj_reverse_step<double>(A, n, slot, (int)(n - n0), pe, ph, grad, s)
                         : adj_reverse_step<float>(A, n, slot, (int)(n - n0), pe, ph, grad, s);
      if (st) return st;
    }
  }
  c->n = A->N;
  return adj_checkpoint(A, A->S, false, s);
}

}  // extern "C"
