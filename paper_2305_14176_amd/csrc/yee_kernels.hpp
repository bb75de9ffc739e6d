// Device kernels of the Yee FDTD step for gfx950 (CDNA4, 64-wide waves).
//
// One leapfrog step (Yee 1966): H^{n+1/2} = H^{n-1/2} - (dt/mu0) curl_e E^n,
// then E^{n+1} = Ca E^n + Cb curl_h H^{n+1/2} (Taflove & Hagness ch. 3), with
// the CPML recursion psi <- b psi + a dF, dF -> dF/kappa + psi inside the
// absorbing layers (Roden & Gedney 2000).  The paper defines no full-wave
// solver; these are the textbook operations.
//
// Fused single pass.  A workgroup owns a tile of TY consecutive y-rows over
// the full x extent and a chunk of z-planes, and marches upward in z.  Each
// row is covered by WPR waves, each lane holding V consecutive x samples; the
// first WPR waves carry the halo row j0-1 (whose H the tile recomputes).  At
// plane k the workgroup
//   1. publishes E^n(k) of its rows in LDS and computes H^{n+1/2}(k) from
//      E^n(k) (x+1 and y+1 neighbours from LDS), E^n(k+1) and H^{n-1/2}(k);
//   2. publishes H^{n+1/2}(k) in LDS and computes E^{n+1}(k) from it (x-1 and
//      y-1 neighbours from LDS) and H^{n+1/2}(k-1) (kept in registers);
//   3. stores both.
// E, H and the H-side psi are ping-ponged, so a tile that recomputes its
// neighbour's halo row reads old values only.
//
// Memory pipelining.  gfx9 counts outstanding vector loads in one in-order
// counter, so waiting for any load also waits for every load issued before
// it.  Each iteration therefore issues its small loads (CPML auxiliaries,
// material and mask data) first and the plane prefetches (E^n(k+2),
// H^{n-1/2}(k+1)) last; waits for the small loads then leave the prefetches
// in flight for a whole iteration.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace yee {

constexpr int kWave = 64;
constexpr int kMaxBlockWaves = 16;   // 1024 threads

// Waves a workgroup may hold at V samples per lane (bounds the registers the
// compiler may give each lane).
__host__ __device__ constexpr int max_block_waves(int V) { return V >= 4 ? 8 : 16; }
constexpr int kMaxSources = 8;

// psi array order (E side in place; H side ping-ponged)
enum { PEXY = 0, PEXZ, PEYZ, PEYX, PEZX, PEZY };
enum { PHXY = 0, PHXZ, PHYZ, PHYX, PHZX, PHZY };

struct SrcDev {
  int32_t comp, i, j, k, kind, pad;
  double amp, t0, tau, f0;
};

template <class C>
struct Coef2 {
  C ca, cb;
};

// Kernel arguments.  Few base pointers (element offsets are derived in the
// kernel) keep the scalar register file from spilling.
template <class T, class C>
struct StepArgs {
  const T* fin;             // E^n, H^{n-1/2}: component c (Ex..Hz) at fin + c * cstride
  T* fout;                  // E^{n+1}, H^{n+1/2}
  uint64_t cstride;         // elements between components
  C* pse;                   // E-side psi, updated in place
  const C* psh_in;          // H-side psi, old
  C* psh_out;               // H-side psi, new
  uint32_t psoff[6];        // element offset of each psi array inside its region
  const C* prof;            // CPML profiles [side E,H][axis][b | a | 1/kappa][plen]
  int32_t plen;
  const int32_t* seg;       // block index per cell: x [px] | y [ny] | z [nz]
  const Coef2<C>* coef;     // (Ca, Cb) per block [nsz][nsy][nsx]
  int32_t nsx, nsxy;
  const int32_t* pec_plane; // [nz], -1 = none
  const uint8_t* pec_mask;  // [nplanes][ny][px], bit 0 Ex, 1 Ey, 2 Ez
  const uint8_t* rowflag;   // [nz][ny], bit 0 source, bit 1 probe
  const int4* probe;        // (comp, i, j, k)
  double* series;           // probe ring [series_len][nprobe]
  int32_t nprobe, series_slot;
  const SrcDev* src;        // soft sources
  int32_t nsrc;
  int64_t n;                // index of the step being taken
  double dt;
  int32_t nx, ny, nz, px;
  int32_t L[3];
  C inv_d[3];
  C dt_mu;
  float enc[6], dec[6];     // FP16 storage scales (2^s, 2^-s)
  int32_t ty, kz, wpr, ny_tiles, ntiles;  // rows per tile, planes per chunk, waves per row
};

// ---------------------------------------------------------------------------
// storage <-> compute conversion
// ---------------------------------------------------------------------------
template <class T, class C>
struct Conv {
  static __device__ __forceinline__ C ld(T v, float) { return static_cast<C>(v); }
  static __device__ __forceinline__ T st(C v, float) { return static_cast<T>(v); }
};
template <>
struct Conv<_Float16, float> {
  static __device__ __forceinline__ float ld(_Float16 v, float dec) { return static_cast<float>(v) * dec; }
  static __device__ __forceinline__ _Float16 st(float v, float enc) { return static_cast<_Float16>(v * enc); }
};

template <class T, int V>
struct alignas(sizeof(T) * V) VecT {
  T v[V];
};

template <class T, class C, int V>
__device__ __forceinline__ void load_row(const T* __restrict__ base, uint32_t off, bool ok, C (&out)[V],
                                         float dec) {
  if (ok) {
    const VecT<T, V> r = *reinterpret_cast<const VecT<T, V>*>(base + off);
#pragma unroll
    for (int e = 0; e < V; ++e) out[e] = Conv<T, C>::ld(r.v[e], dec);
  } else {
#pragma unroll
    for (int e = 0; e < V; ++e) out[e] = C(0);
  }
}

template <class T, class C, int V>
__device__ __forceinline__ void store_row(T* __restrict__ base, uint32_t off, const C (&in)[V], float enc) {
  VecT<T, V> r;
#pragma unroll
  for (int e = 0; e < V; ++e) r.v[e] = Conv<T, C>::st(in[e], enc);
  *reinterpret_cast<VecT<T, V>*>(base + off) = r;
}

// Round a computed value to what storage would hold (identity unless FP16).
template <class T, class C>
__device__ __forceinline__ C to_storage(C v, float enc, float dec) {
  return Conv<T, C>::ld(Conv<T, C>::st(v, enc), dec);
}

// Source waveform in FP64: w(t) = -2u exp(-u^2) or sin(2 pi f0 (t - t0)) exp(-u^2).
__device__ __noinline__ double waveform(const SrcDev s, double t) {
  const double u = (t - s.t0) / s.tau;
  const double g = exp(-u * u);
  if (s.kind == 0) return -2.0 * u * g;
  return sin(2.0 * M_PI * s.f0 * (t - s.t0)) * g;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// LDS footprint of one workgroup in bytes: E rows j0-1..j0+ty and H rows
// j0-1..j0+ty-1, three components of RL = wpr * 64 * V samples each; the
// source values; and per-plane tables of the z-chunk (kz + 1 planes): six z
// profiles, the z block offset, the PEC plane index and the row flags.
__host__ __device__ inline size_t step_lds_bytes_for(int ty, int wpr, int V, int kz, size_t csize) {
  const size_t rl = (size_t)wpr * kWave * V;
  const size_t nk = (size_t)kz + 1;
  size_t b = ((size_t)(ty + 2) * 3 * rl + (size_t)(ty + 1) * 3 * rl + kMaxSources + 6 * nk) * csize;
  b += 2 * nk * sizeof(int32_t);
  b += (size_t)(ty + 1) * nk;
  return (b + 15) & ~size_t(15);
}

// Per-lane data of one plane that is small but still comes from memory: CPML
// auxiliaries (H side old, E side in place), the material coefficients and
// the PEC mask.  It is loaded one plane ahead of its use.
template <class C, int V>
struct PlaneAux {
  C ph[6][V];   // H-side psi, PH* order
  C pe[6][V];   // E-side psi, PE* order
  Coef2<C> cf[V];
  uint32_t pm[V];
};

// ---------------------------------------------------------------------------
// The fused step kernel
// ---------------------------------------------------------------------------
// One tile (ytile, chunk) of one grid.  Waves beyond (ty + 1) * wpr (spare
// waves of a fixed-size workgroup) take part in the barriers only.
template <class T, class C, int V>
__device__ __forceinline__ void step_tile(const StepArgs<T, C>& a, const int ytile, const int chunk,
                                          unsigned char* smem_raw) {
  const int wpr = a.wpr;
  const int RL = wpr * kWave * V;                 // LDS row length
  const int nk1 = a.kz + 1;                       // stride of the per-plane tables
  C* ldsE = reinterpret_cast<C*>(smem_raw);      // [(ty+2)][3][RL]: E^n(k) rows j0-1..j0+ty
  C* ldsH = ldsE + (a.ty + 2) * 3 * RL;           // [(ty+1)][3][RL]: H^{n+1/2}(k) rows j0-1..j0+ty-1
  C* ldsS = ldsH + (a.ty + 1) * 3 * RL;           // [kMaxSources]: amp * w((n+1) dt)
  C* tzp = ldsS + kMaxSources;                    // [6][nk1]: z profiles bE aE kE bH aH kH
  int32_t* tzs = reinterpret_cast<int32_t*>(tzp + 6 * nk1);  // [nk1]: z block index * nsx * nsy
  int32_t* tzl = tzs + nk1;                       // [nk1]: PEC plane index
  uint8_t* tfl = reinterpret_cast<uint8_t*>(tzl + nk1);      // [ty+1][nk1]: row flags

  const int nx = a.nx, ny = a.ny, nz = a.nz, px = a.px;
  const int Lx = a.L[0], Ly = a.L[1], Lz = a.L[2];
  const int j0 = ytile * a.ty;
  const int k0 = chunk * a.kz;
  const int k1 = min(nz, k0 + a.kz);
  const int kstart = k0 > 0 ? k0 - 1 : 0;
  const int nk = k1 - kstart;

  // ---- per-workgroup tables (sources and the chunk's planes) ----
  if ((int)threadIdx.x < a.nsrc) {
    const SrcDev sd = a.src[threadIdx.x];
    ldsS[threadIdx.x] = static_cast<C>(sd.amp * waveform(sd, (double)(a.n + 1) * a.dt));
  }
  for (int q = threadIdx.x; q < nk; q += blockDim.x) {
    const int k = kstart + q;
    const bool inz = (k < Lz || k >= nz - Lz);
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int side = u / 3, qq = u % 3;   // b, a, 1/kappa of the E and H side
      tzp[u * nk1 + q] = inz ? a.prof[((side * 3 + 2) * 3 + qq) * a.plen + k] : (qq == 1 ? C(0) : C(1));
    }
    tzs[q] = a.seg[px + ny + k] * a.nsxy;
    tzl[q] = a.pec_plane[k];
  }
  for (int q = threadIdx.x; q < (a.ty + 1) * nk; q += blockDim.x) {
    const int rr = q / nk, kk = q - rr * nk;
    const int jj = j0 - 1 + rr;
    tfl[rr * nk1 + kk] = (jj >= 0 && jj < ny) ? a.rowflag[(uint32_t)(kstart + kk) * ny + jj] : 0;
  }
  __syncthreads();

  const int wv = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const bool dummy = wv >= (a.ty + 1) * wpr;  // spare wave: barriers only
  const int r = dummy ? 0 : wv / wpr;     // tile row: 0 = halo row j0-1
  const int xs = dummy ? 0 : wv - r * wpr;  // x segment of the row
  const int j = j0 - 1 + r;
  const bool halo = !dummy && (r == 0);
  const bool row_ok = !dummy && (j >= 0) && (j < ny);
  const int jc = min(max(j, 0), ny - 1);
  const int xl = (xs * kWave + lane) * V;  // first sample of the lane within the row
  const bool lane_ok = xl < nx;
  const bool ld_ok = row_ok && lane_ok;
  const bool own = !halo && ld_ok;
  const uint32_t plane = (uint32_t)ny * (uint32_t)px;
  const uint32_t rowoff = (uint32_t)jc * (uint32_t)px + (uint32_t)xl;
  const C idx_ = a.inv_d[0], idy = a.inv_d[1], idz = a.inv_d[2];
  const uint64_t cs = a.cstride;
  const T* __restrict__ fEx = a.fin;
  const T* __restrict__ fEy = a.fin + cs;
  const T* __restrict__ fEz = a.fin + 2 * cs;
  const T* __restrict__ fHx = a.fin + 3 * cs;
  const T* __restrict__ fHy = a.fin + 4 * cs;
  const T* __restrict__ fHz = a.fin + 5 * cs;

  bool xin[V];
#pragma unroll
  for (int e = 0; e < V; ++e) xin[e] = (xl + e) < nx;

  const bool iny = row_ok && (j < Ly || j >= ny - Ly);
  const int sy = j < Ly ? j : j - ny + 2 * Ly;
  // x-layer membership and the lane's constant x profiles (E and H side)
  bool inx[V];
  int sxv[V];
  C bxe[V], axe[V], kxe[V], bxh[V], axh[V], kxh[V];
  bool lane_inx = false;
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const int i = xl + e;
    inx[e] = row_ok && xin[e] && (i < Lx || i >= nx - Lx);
    sxv[e] = i < Lx ? i : i - nx + 2 * Lx;
    bxe[e] = C(1); axe[e] = C(0); kxe[e] = C(1); bxh[e] = C(1); axh[e] = C(0); kxh[e] = C(1);
    if (inx[e]) {
      bxe[e] = a.prof[(0 * 3 + 0) * a.plen + i];
      axe[e] = a.prof[(0 * 3 + 1) * a.plen + i];
      kxe[e] = a.prof[(0 * 3 + 2) * a.plen + i];
      bxh[e] = a.prof[(9 + 0) * a.plen + i];
      axh[e] = a.prof[(9 + 1) * a.plen + i];
      kxh[e] = a.prof[(9 + 2) * a.plen + i];
    }
    lane_inx = lane_inx || inx[e];
  }
  // y profiles (uniform over the row)
  C bye = 1, aye = 0, kye = 1, byh = 1, ayh = 0, kyh = 1;
  if (iny) {
    bye = a.prof[(3 + 0) * a.plen + j]; aye = a.prof[(3 + 1) * a.plen + j]; kye = a.prof[(3 + 2) * a.plen + j];
    byh = a.prof[(12 + 0) * a.plen + j]; ayh = a.prof[(12 + 1) * a.plen + j]; kyh = a.prof[(12 + 2) * a.plen + j];
  }
  int segxy[V];
#pragma unroll
  for (int e = 0; e < V; ++e) segxy[e] = (xin[e] ? a.seg[xl + e] : 0) + a.seg[px + jc] * a.nsx;

  // Small per-lane data of plane k (into aux): issued ahead of the plane prefetch.
  auto load_aux = [&](int k, PlaneAux<C, V>& x) {
    const bool upd = (k >= k0) && own;
    const bool inz = row_ok && (k < Lz || k >= nz - Lz);
    const int sz = k < Lz ? k : k - nz + 2 * Lz;
    const uint32_t qy = ((uint32_t)k * (2 * Ly) + sy) * px + xl;
    const uint32_t qz = ((uint32_t)sz * ny + jc) * px + xl;
    const uint32_t qx = ((uint32_t)k * ny + jc) * (2 * Lx);
#pragma unroll
    for (int e = 0; e < V; ++e) {
#pragma unroll
      for (int u = 0; u < 6; ++u) { x.ph[u][e] = C(0); x.pe[u][e] = C(0); }
      x.pm[e] = 0;
    }
    if (iny) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        if (!xin[e]) continue;
        x.ph[PHXY][e] = a.psh_in[a.psoff[PHXY] + qy + e];
        x.ph[PHZY][e] = a.psh_in[a.psoff[PHZY] + qy + e];
        if (upd) { x.pe[PEXY][e] = a.pse[a.psoff[PEXY] + qy + e]; x.pe[PEZY][e] = a.pse[a.psoff[PEZY] + qy + e]; }
      }
    }
    if (inz) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        if (!xin[e]) continue;
        x.ph[PHXZ][e] = a.psh_in[a.psoff[PHXZ] + qz + e];
        x.ph[PHYZ][e] = a.psh_in[a.psoff[PHYZ] + qz + e];
        if (upd) { x.pe[PEXZ][e] = a.pse[a.psoff[PEXZ] + qz + e]; x.pe[PEYZ][e] = a.pse[a.psoff[PEYZ] + qz + e]; }
      }
    }
    if (lane_inx) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        if (!inx[e]) continue;
        x.ph[PHYX][e] = a.psh_in[a.psoff[PHYX] + qx + sxv[e]];
        x.ph[PHZX][e] = a.psh_in[a.psoff[PHZX] + qx + sxv[e]];
        if (upd) { x.pe[PEYX][e] = a.pse[a.psoff[PEYX] + qx + sxv[e]]; x.pe[PEZX][e] = a.pse[a.psoff[PEZX] + qx + sxv[e]]; }
      }
    }
    const int zs = tzs[k - kstart];
#pragma unroll
    for (int e = 0; e < V; ++e) x.cf[e] = a.coef[segxy[e] + zs];
    const int pl = tzl[k - kstart];
    if (pl >= 0 && own) {
#pragma unroll
      for (int e = 0; e < V; ++e) x.pm[e] = a.pec_mask[((uint32_t)pl * ny + jc) * px + xl + e];
    }
  };

  // Software pipeline over the z-march: at plane k the registers hold E^n(k),
  // E^n(k+1), H^{n-1/2}(k), the plane's small data (cur) and, in the halo
  // waves, Ez/Ex of the row above the tile at plane k.
  C ec[3][V], en[3][V], hc[3][V], tz[V], tx[V];
  PlaneAux<C, V> cur;
  const int jt = j0 + a.ty;  // row above the tile
  const bool top_ok = halo && lane_ok && jt < ny;
  const uint32_t rowoff_t = (uint32_t)min(jt, ny - 1) * (uint32_t)px + (uint32_t)xl;
  {
    load_aux(kstart, cur);
    const uint32_t off = (uint32_t)kstart * plane + rowoff;
    const bool ok1 = ld_ok && (kstart + 1 < nz);
    load_row<T, C, V>(fEx, off, ld_ok, ec[0], a.dec[0]);
    load_row<T, C, V>(fEy, off, ld_ok, ec[1], a.dec[1]);
    load_row<T, C, V>(fEz, off, ld_ok, ec[2], a.dec[2]);
    load_row<T, C, V>(fEx, off + plane, ok1, en[0], a.dec[0]);
    load_row<T, C, V>(fEy, off + plane, ok1, en[1], a.dec[1]);
    load_row<T, C, V>(fEz, off + plane, ok1, en[2], a.dec[2]);
    load_row<T, C, V>(fHx, off, ld_ok, hc[0], a.dec[3]);
    load_row<T, C, V>(fHy, off, ld_ok && !halo, hc[1], a.dec[4]);
    load_row<T, C, V>(fHz, off, ld_ok, hc[2], a.dec[5]);
    const uint32_t offt = (uint32_t)kstart * plane + rowoff_t;
    load_row<T, C, V>(fEz, offt, top_ok, tz, a.dec[2]);
    load_row<T, C, V>(fEx, offt, top_ok, tx, a.dec[0]);
  }
  C hxp[V], hyp[V];  // H^{n+1/2}(k-1), own row
#pragma unroll
  for (int e = 0; e < V; ++e) { hxp[e] = C(0); hyp[e] = C(0); }

  C* rowE = ldsE + r * 3 * RL;        // own row in the E buffer
  C* rowH = ldsH + r * 3 * RL;        // own row in the H buffer

  // One plane of the march.  The registers of the plane prefetch come in two
  // sets used alternately (en/hc/aux/tz of this plane, the other set filled
  // for the next one), so no register whose load is still in flight is ever
  // copied; the march is unrolled by two to alternate them.
  auto plane_step = [&](const int k, C (&en)[3][V], C (&en2)[3][V], C (&hc)[3][V], C (&hn)[3][V],
                        PlaneAux<C, V>& cur, PlaneAux<C, V>& nxt, C (&tz)[V], C (&tx)[V], C (&tzn)[V],
                        C (&txn)[V]) {
    const bool active = k >= k0;
    const bool more = k + 1 < k1;  // another plane follows in this chunk
    const uint32_t off = (uint32_t)k * plane + rowoff;
    const int kq = k - kstart;
    const bool inz = row_ok && (k < Lz || k >= nz - Lz);
    const int sz = k < Lz ? k : k - nz + 2 * Lz;
    const bool upd = active && own;
    const uint32_t qy = ((uint32_t)k * (2 * Ly) + sy) * px + xl;
    const uint32_t qz = ((uint32_t)sz * ny + jc) * px + xl;
    const uint32_t qx = ((uint32_t)k * ny + jc) * (2 * Lx);

    // ---- 1. loads for the next iterations: small data of plane k+1 first,
    //         then E^n(k+2), H^{n-1/2}(k+1) and the next row above ----
    if (more) load_aux(k + 1, nxt);
    __builtin_amdgcn_sched_barrier(0);
    {
      const bool ok2 = ld_ok && more && (k + 2 < nz);
      const bool okh = ld_ok && more;
      load_row<T, C, V>(fEx, off + 2 * plane, ok2, en2[0], a.dec[0]);
      load_row<T, C, V>(fEy, off + 2 * plane, ok2, en2[1], a.dec[1]);
      load_row<T, C, V>(fEz, off + 2 * plane, ok2, en2[2], a.dec[2]);
      load_row<T, C, V>(fHx, off + plane, okh, hn[0], a.dec[3]);
      load_row<T, C, V>(fHy, off + plane, okh && !halo, hn[1], a.dec[4]);
      load_row<T, C, V>(fHz, off + plane, okh, hn[2], a.dec[5]);
      const uint32_t offt = (uint32_t)(k + 1) * plane + rowoff_t;
      load_row<T, C, V>(fEz, offt, top_ok && more, tzn, a.dec[2]);
      load_row<T, C, V>(fEx, offt, top_ok && more, txn, a.dec[0]);
    }
    __builtin_amdgcn_sched_barrier(0);

    // ---- 2. publish E^n(k) ----
    if (!dummy) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        rowE[xl + e] = ec[0][e];
        rowE[RL + xl + e] = ec[1][e];
        rowE[2 * RL + xl + e] = ec[2][e];
      }
    }
    if (halo) {
      C* rt = ldsE + (a.ty + 1) * 3 * RL;
#pragma unroll
      for (int e = 0; e < V; ++e) { rt[xl + e] = tx[e]; rt[2 * RL + xl + e] = tz[e]; }
    }
    __syncthreads();

    // ---- 3. H half step at plane k ----
    const C bze = tzp[0 * nk1 + kq], aze = tzp[1 * nk1 + kq], kze = tzp[2 * nk1 + kq];
    const C bzh = tzp[3 * nk1 + kq], azh = tzp[4 * nk1 + kq], kzh = tzp[5 * nk1 + kq];
    C hx[V], hy[V], hz[V];
    {
      const C* up = rowE + 3 * RL;   // row j+1
      C ezu[V], exu[V], ezr[V], eyr[V];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        exu[e] = up[xl + e];
        ezu[e] = up[2 * RL + xl + e];
      }
#pragma unroll
      for (int e = 0; e < V - 1; ++e) { eyr[e] = ec[1][e + 1]; ezr[e] = ec[2][e + 1]; }
      {
        const int ir = xl + V;  // x+1 neighbour of the last sample (0 beyond the grid)
        const bool okr = ir < nx;
        eyr[V - 1] = okr ? rowE[RL + min(ir, RL - 1)] : C(0);
        ezr[V - 1] = okr ? rowE[2 * RL + min(ir, RL - 1)] : C(0);
      }
#pragma unroll
      for (int e = 0; e < V; ++e) {
        C dEz_dy = (ezu[e] - ec[2][e]) * idy;
        C dEy_dz = (en[1][e] - ec[1][e]) * idz;
        C dEx_dz = (en[0][e] - ec[0][e]) * idz;
        C dEz_dx = (ezr[e] - ec[2][e]) * idx_;
        C dEy_dx = (eyr[e] - ec[1][e]) * idx_;
        C dEx_dy = (exu[e] - ec[0][e]) * idy;
        if (iny) {
          cur.ph[PHXY][e] = byh * cur.ph[PHXY][e] + ayh * dEz_dy;
          cur.ph[PHZY][e] = byh * cur.ph[PHZY][e] + ayh * dEx_dy;
          dEz_dy = kyh * dEz_dy + cur.ph[PHXY][e];
          dEx_dy = kyh * dEx_dy + cur.ph[PHZY][e];
        }
        if (inz) {
          cur.ph[PHXZ][e] = bzh * cur.ph[PHXZ][e] + azh * dEy_dz;
          cur.ph[PHYZ][e] = bzh * cur.ph[PHYZ][e] + azh * dEx_dz;
          dEy_dz = kzh * dEy_dz + cur.ph[PHXZ][e];
          dEx_dz = kzh * dEx_dz + cur.ph[PHYZ][e];
        }
        if (inx[e]) {
          cur.ph[PHYX][e] = bxh[e] * cur.ph[PHYX][e] + axh[e] * dEz_dx;
          cur.ph[PHZX][e] = bxh[e] * cur.ph[PHZX][e] + axh[e] * dEy_dx;
          dEz_dx = kxh[e] * dEz_dx + cur.ph[PHYX][e];
          dEy_dx = kxh[e] * dEy_dx + cur.ph[PHZX][e];
        }
        const bool ok = row_ok && xin[e];
        hx[e] = ok ? to_storage<T, C>(hc[0][e] - a.dt_mu * (dEz_dy - dEy_dz), a.enc[3], a.dec[3]) : C(0);
        hy[e] = ok ? to_storage<T, C>(hc[1][e] - a.dt_mu * (dEx_dz - dEz_dx), a.enc[4], a.dec[4]) : C(0);
        hz[e] = ok ? to_storage<T, C>(hc[2][e] - a.dt_mu * (dEy_dx - dEx_dy), a.enc[5], a.dec[5]) : C(0);
      }
    }

    // ---- 4. publish H^{n+1/2}(k) ----
    if (!dummy) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        rowH[xl + e] = hx[e];
        rowH[RL + xl + e] = hy[e];
        rowH[2 * RL + xl + e] = hz[e];
      }
    }
    __syncthreads();

    // ---- 5. E half step at plane k (own rows) and stores ----
    if (upd) {
      // H-side psi of the own row
      if (iny) {
#pragma unroll
        for (int e = 0; e < V; ++e)
          if (xin[e]) {
            a.psh_out[a.psoff[PHXY] + qy + e] = cur.ph[PHXY][e];
            a.psh_out[a.psoff[PHZY] + qy + e] = cur.ph[PHZY][e];
          }
      }
      if (inz) {
#pragma unroll
        for (int e = 0; e < V; ++e)
          if (xin[e]) {
            a.psh_out[a.psoff[PHXZ] + qz + e] = cur.ph[PHXZ][e];
            a.psh_out[a.psoff[PHYZ] + qz + e] = cur.ph[PHYZ][e];
          }
      }
      if (lane_inx) {
#pragma unroll
        for (int e = 0; e < V; ++e)
          if (inx[e]) {
            a.psh_out[a.psoff[PHYX] + qx + sxv[e]] = cur.ph[PHYX][e];
            a.psh_out[a.psoff[PHZX] + qx + sxv[e]] = cur.ph[PHZX][e];
          }
      }
      const C* dn = rowH - 3 * RL;   // row j-1
      C hxd[V], hzd[V], hyl[V], hzl[V];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        hxd[e] = dn[xl + e];
        hzd[e] = dn[2 * RL + xl + e];
      }
#pragma unroll
      for (int e = 1; e < V; ++e) { hyl[e] = hy[e - 1]; hzl[e] = hz[e - 1]; }
      {
        const int il = max(xl - 1, 0);   // x-1 neighbour of the first sample (unused at i = 0)
        hyl[0] = rowH[RL + il];
        hzl[0] = rowH[2 * RL + il];
      }
      C exo[V], eyo[V], ezo[V];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const int i = xl + e;
        C dHz_dy = (hz[e] - hzd[e]) * idy;
        C dHy_dz = (hy[e] - hyp[e]) * idz;
        C dHx_dz = (hx[e] - hxp[e]) * idz;
        C dHz_dx = (hz[e] - hzl[e]) * idx_;
        C dHy_dx = (hy[e] - hyl[e]) * idx_;
        C dHx_dy = (hx[e] - hxd[e]) * idy;
        // tangential E on the outer faces is never updated
        const bool ux = (j > 0) && (k > 0) && xin[e];
        const bool uy = (i > 0) && (k > 0) && xin[e];
        const bool uz = (i > 0) && (j > 0) && xin[e];
        if (iny) {
          cur.pe[PEXY][e] = bye * cur.pe[PEXY][e] + aye * dHz_dy;
          cur.pe[PEZY][e] = bye * cur.pe[PEZY][e] + aye * dHx_dy;
          dHz_dy = kye * dHz_dy + cur.pe[PEXY][e];
          dHx_dy = kye * dHx_dy + cur.pe[PEZY][e];
        }
        if (inz) {
          cur.pe[PEXZ][e] = bze * cur.pe[PEXZ][e] + aze * dHy_dz;
          cur.pe[PEYZ][e] = bze * cur.pe[PEYZ][e] + aze * dHx_dz;
          dHy_dz = kze * dHy_dz + cur.pe[PEXZ][e];
          dHx_dz = kze * dHx_dz + cur.pe[PEYZ][e];
        }
        if (inx[e]) {
          cur.pe[PEYX][e] = bxe[e] * cur.pe[PEYX][e] + axe[e] * dHz_dx;
          cur.pe[PEZX][e] = bxe[e] * cur.pe[PEZX][e] + axe[e] * dHy_dx;
          dHz_dx = kxe[e] * dHz_dx + cur.pe[PEYX][e];
          dHy_dx = kxe[e] * dHy_dx + cur.pe[PEZX][e];
        }
        const C ca = cur.cf[e].ca, cb = cur.cf[e].cb;
        const uint32_t m = cur.pm[e];
        const C cax = (m & 1) ? C(0) : ca, cbx = (m & 1) ? C(0) : cb;
        const C cay = (m & 2) ? C(0) : ca, cby = (m & 2) ? C(0) : cb;
        const C caz = (m & 4) ? C(0) : ca, cbz = (m & 4) ? C(0) : cb;
        exo[e] = ux ? cax * ec[0][e] + cbx * (dHz_dy - dHy_dz) : ec[0][e];
        eyo[e] = uy ? cay * ec[1][e] + cby * (dHx_dz - dHz_dx) : ec[1][e];
        ezo[e] = uz ? caz * ec[2][e] + cbz * (dHy_dx - dHx_dy) : ec[2][e];
        // E-side psi of the updated samples (wall samples keep 0)
        if (!ux) { cur.pe[PEXY][e] = C(0); cur.pe[PEXZ][e] = C(0); }
        if (!uy) { cur.pe[PEYZ][e] = C(0); cur.pe[PEYX][e] = C(0); }
        if (!uz) { cur.pe[PEZX][e] = C(0); cur.pe[PEZY][e] = C(0); }
      }
      if (iny) {
#pragma unroll
        for (int e = 0; e < V; ++e)
          if (xin[e]) {
            a.pse[a.psoff[PEXY] + qy + e] = cur.pe[PEXY][e];
            a.pse[a.psoff[PEZY] + qy + e] = cur.pe[PEZY][e];
          }
      }
      if (inz) {
#pragma unroll
        for (int e = 0; e < V; ++e)
          if (xin[e]) {
            a.pse[a.psoff[PEXZ] + qz + e] = cur.pe[PEXZ][e];
            a.pse[a.psoff[PEYZ] + qz + e] = cur.pe[PEYZ][e];
          }
      }
      if (lane_inx) {
#pragma unroll
        for (int e = 0; e < V; ++e)
          if (inx[e]) {
            a.pse[a.psoff[PEYX] + qx + sxv[e]] = cur.pe[PEYX][e];
            a.pse[a.psoff[PEZX] + qx + sxv[e]] = cur.pe[PEZX][e];
          }
      }
      const uint8_t flags = tfl[r * nk1 + kq];
      if (flags & 1) {
        for (int s = 0; s < a.nsrc; ++s) {
          const SrcDev sp = a.src[s];
          if (sp.j == j && sp.k == k) {
            const C v = ldsS[s];
#pragma unroll
            for (int e = 0; e < V; ++e) {
              if (xl + e == sp.i) {
                if (sp.comp == 0) exo[e] += v;
                else if (sp.comp == 1) eyo[e] += v;
                else ezo[e] += v;
              }
            }
          }
        }
      }
#pragma unroll
      for (int e = 0; e < V; ++e) {
        exo[e] = to_storage<T, C>(exo[e], a.enc[0], a.dec[0]);
        eyo[e] = to_storage<T, C>(eyo[e], a.enc[1], a.dec[1]);
        ezo[e] = to_storage<T, C>(ezo[e], a.enc[2], a.dec[2]);
      }
      store_row<T, C, V>(a.fout, off, exo, a.enc[0]);
      store_row<T, C, V>(a.fout + cs, off, eyo, a.enc[1]);
      store_row<T, C, V>(a.fout + 2 * cs, off, ezo, a.enc[2]);
      store_row<T, C, V>(a.fout + 3 * cs, off, hx, a.enc[3]);
      store_row<T, C, V>(a.fout + 4 * cs, off, hy, a.enc[4]);
      store_row<T, C, V>(a.fout + 5 * cs, off, hz, a.enc[5]);
      if (flags & 2) {
        for (int p = 0; p < a.nprobe; ++p) {
          const int4 pr = a.probe[p];
          if (pr.z == j && pr.w == k) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
              if (xl + e == pr.y) {
                const C v = pr.x == 0 ? exo[e] : pr.x == 1 ? eyo[e] : pr.x == 2 ? ezo[e]
                          : pr.x == 3 ? hx[e] : pr.x == 4 ? hy[e] : hz[e];
                a.series[(size_t)a.series_slot * a.nprobe + p] = static_cast<double>(v);
              }
            }
          }
        }
      }
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
      hxp[e] = hx[e];
      hyp[e] = hy[e];
#pragma unroll
      for (int c = 0; c < 3; ++c) ec[c][e] = en[c][e];   // E^n(k+1) has arrived: it was used above
    }
  };

  C en_b[3][V], hc_b[3][V], tz_b[V], tx_b[V];
  PlaneAux<C, V> aux_b;
  for (int k = kstart; k < k1; k += 2) {
    plane_step(k, en, en_b, hc, hc_b, cur, aux_b, tz, tx, tz_b, tx_b);
    if (k + 1 < k1) plane_step(k + 1, en_b, en, hc_b, hc, aux_b, cur, tz_b, tx_b, tz, tx);
  }
}

// ---------------------------------------------------------------------------
// The fused step kernel: one grid, one tile per workgroup.
// ---------------------------------------------------------------------------
template <class T, class C, int V>
__global__ void __launch_bounds__(kWave * max_block_waves(V))
step_kernel(const StepArgs<T, C> a) {
  extern __shared__ unsigned char smem_raw[];
  // XCD-aware tile order: consecutive workgroup ids are dealt round-robin to
  // the 8 XCDs, so give each XCD a contiguous run of tiles (neighbouring
  // y-tiles of one z-chunk share halo rows in that XCD's L2).
  const int per_xcd = gridDim.x >> 3;
  const int t = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (t >= a.ntiles) return;
  step_tile<T, C, V>(a, t % a.ny_tiles, t / a.ny_tiles, smem_raw);
}

// ---------------------------------------------------------------------------
// Batched stepper: many grids ("slots") per launch.  The host writes one
// descriptor per slot (its static arguments, both field / psi sets, the steps
// already taken and the steps requested) before a replay; a replay is a
// sequence of launches with step offsets q = 0, 1, ... (captured once in a
// HIP graph).  Workgroups stride over the global tile list of all slots, so
// the grid size is fixed while slots come and go between replays; a slot whose
// request is complete skips its tiles.
// ---------------------------------------------------------------------------
template <class T, class C>
struct SlotDesc {
  StepArgs<T, C> a;         // static arguments; fin/fout/psh/n/series_slot are set per step
  const T* set[2];          // field sets (E, H ping-pong)
  C* psh[2];                // H-side psi sets
  int64_t base_n;           // steps taken before this replay
  int64_t n_end;            // steps requested
  int32_t series_len;
  int32_t tile0;            // first global tile of the slot
  int32_t pad[2];
};

template <class T, class C, int V>
__global__ void __launch_bounds__(kWave * max_block_waves(V))
batch_step_kernel(const SlotDesc<T, C>* __restrict__ slots, const int32_t* __restrict__ hdr, const int q) {
  extern __shared__ unsigned char smem_raw[];
  const int nslots = hdr[0], total = hdr[1];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int s = 0;
    while (s + 1 < nslots && slots[s + 1].tile0 <= t) ++s;
    const int64_t n = slots[s].base_n + q;
    if (n < slots[s].n_end) {
      StepArgs<T, C> a = slots[s].a;
      const int par = (int)(n & 1);
      a.fin = slots[s].set[par];
      a.fout = const_cast<T*>(slots[s].set[par ^ 1]);
      a.psh_in = slots[s].psh[par];
      a.psh_out = slots[s].psh[par ^ 1];
      a.n = n;
      a.series_slot = (int32_t)(n % slots[s].series_len);
      const int tl = t - slots[s].tile0;
      step_tile<T, C, V>(a, tl % a.ny_tiles, tl / a.ny_tiles, smem_raw);
    }
    __syncthreads();  // the next tile reuses the LDS
  }
}

// ---------------------------------------------------------------------------
// Running DFT fold: one wave per (probe, frequency); lanes stride over the
// samples of the chunk, partial sums meet in a butterfly of lane shuffles.
// X_p(f) += sum_n y_p[n] exp(-i 2 pi f n dt) dt for n = n_first .. n_first+count-1.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256)
dft_fold_kernel(const double* __restrict__ series, int nprobe, int series_len, int64_t n_first,
                int count, const double* __restrict__ freqs, int nf, double dt,
                double2* __restrict__ acc) {
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wid >= nprobe * nf) return;
  const int p = wid / nf;
  const int m = wid % nf;
  const double fdt = freqs[m] * dt;
  double re = 0.0, im = 0.0;
  for (int s = lane; s < count; s += kWave) {
    const int64_t n = n_first + s;                  // 1-based step number
    const double y = series[(size_t)((n - 1) % series_len) * nprobe + p];
    double ph = fdt * (double)n;                    // cycles
    ph -= floor(ph);
    double sn, cs;
    sincospi(2.0 * ph, &sn, &cs);
    re += y * cs;
    im -= y * sn;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    re += __shfl_xor(re, o, kWave);
    im += __shfl_xor(im, o, kWave);
  }
  if (lane == 0) {
    double2 v = acc[wid];
    v.x += re * dt;
    v.y += im * dt;
    acc[wid] = v;
  }
}

}  // namespace yee
