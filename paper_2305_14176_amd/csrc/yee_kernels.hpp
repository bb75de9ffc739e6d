// Device kernels of the Yee FDTD step for gfx950 (CDNA4, 64-wide waves).
//
// One leapfrog step (Yee 1966): H^{n+1/2} = H^{n-1/2} - (dt/mu0) curl_e E^n,
// then E^{n+1} = Ca E^n + Cb curl_h H^{n+1/2} (Taflove & Hagness ch. 3), with
// the CPML recursion psi <- b psi + a dF, dF -> dF/kappa + psi inside the
// absorbing layers (Roden & Gedney 2000).  The paper defines no full-wave
// solver; these are the textbook operations.
//
// Fused single pass.  A workgroup owns a tile of TY consecutive y-rows (full
// x extent: one wave per row, V consecutive x samples per lane) and a chunk
// of z-planes, and marches upward in z.  At plane k it
//   1. computes H^{n+1/2}(k) for its rows plus the halo row j0-1 (wave 0),
//      from E^n(k), E^n(k+1) and H^{n-1/2}(k);
//   2. computes E^{n+1}(k) from H^{n+1/2}(k) (rows j, j-1 via LDS; x-1 via a
//      lane shuffle) and H^{n+1/2}(k-1) (kept in registers);
//   3. stores both.
// y-neighbours move through LDS, x-neighbours through lane shuffles, z-
// neighbours stay in registers.  E, H and the H-side psi are ping-ponged so a
// tile that recomputes its neighbour's halo row reads the old values.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace yee {

constexpr int kWave = 64;
constexpr int kMaxTileRows = 7;

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

template <class T, class C>
struct StepArgs {
  const T* e_in[3];
  const T* h_in[3];
  T* e_out[3];
  T* h_out[3];
  C* psi_e[6];
  const C* psi_h_in[6];
  C* psi_h_out[6];
  // CPML profiles per side (0 = E, 1 = H) and axis: b, a, 1/kappa over the axis
  const C* pb[2][3];
  const C* pa[2][3];
  const C* pk[2][3];
  // materials
  const int32_t* segx;  // [px]
  const int32_t* segy;  // [ny]
  const int32_t* segz;  // [nz]
  const Coef2<C>* coef; // [nsz][nsy][nsx]
  int32_t nsx, nsxy;
  // PEC planes
  const int32_t* pec_plane;  // [nz], -1 = none
  const uint8_t* pec_mask;   // [nplanes][ny][px]
  // sources / probes
  const uint8_t* rowflag;    // [nz][ny] bit0 source, bit1 probe
  const SrcDev* src;
  int32_t nsrc;
  const int4* probe;         // (comp, i, j, k)
  int32_t nprobe;
  double* series;            // [series_len][nprobe]
  int32_t series_len;
  // geometry
  int32_t nx, ny, nz, px;
  int32_t L[3];
  C inv_d[3];
  C dt_mu;
  double dt;
  int64_t n;                 // index of the step being taken
  float enc[6], dec[6];      // FP16 storage scales (2^s, 2^-s)
  // launch shape
  int32_t ty, kz, ny_tiles, ntiles;
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
__device__ __forceinline__ void load_row(const T* __restrict__ p, bool ok, C (&out)[V], float dec) {
  if (ok) {
    const VecT<T, V> r = *reinterpret_cast<const VecT<T, V>*>(p);
#pragma unroll
    for (int e = 0; e < V; ++e) out[e] = Conv<T, C>::ld(r.v[e], dec);
  } else {
#pragma unroll
    for (int e = 0; e < V; ++e) out[e] = C(0);
  }
}

template <class T, class C, int V>
__device__ __forceinline__ void store_row(T* __restrict__ p, const C (&in)[V], float enc) {
  VecT<T, V> r;
#pragma unroll
  for (int e = 0; e < V; ++e) r.v[e] = Conv<T, C>::st(in[e], enc);
  *reinterpret_cast<VecT<T, V>*>(p) = r;
}

// Round a computed value to what storage would hold (identity unless FP16).
template <class T, class C>
__device__ __forceinline__ C to_storage(C v, float enc, float dec) {
  return Conv<T, C>::ld(Conv<T, C>::st(v, enc), dec);
}

// Source waveform in FP64 (same definitions as the header documents).
__device__ __forceinline__ double waveform(const SrcDev& s, double t) {
  const double u = (t - s.t0) / s.tau;
  const double g = exp(-u * u);
  if (s.kind == 0) return -2.0 * u * g;
  return sin(2.0 * M_PI * s.f0 * (t - s.t0)) * g;
}

template <class C>
__device__ __forceinline__ C shfl_down1(C v, int lane) {
  C r = __shfl_down(v, 1, kWave);
  return lane == kWave - 1 ? C(0) : r;
}
template <class C>
__device__ __forceinline__ C shfl_up1(C v, int lane) {
  C r = __shfl_up(v, 1, kWave);
  return lane == 0 ? C(0) : r;
}

// ---------------------------------------------------------------------------
// The fused step kernel
// ---------------------------------------------------------------------------
template <class T, class C, int V>
__global__ void __launch_bounds__(kWave * (kMaxTileRows + 1))
step_kernel(const StepArgs<T, C> a) {
  extern __shared__ unsigned char smem_raw[];
  constexpr int RW = kWave * V;
  C* ldsE = reinterpret_cast<C*>(smem_raw);      // [(ty+2)][2][RW]: Ez, Ex at plane k
  C* ldsH = ldsE + (a.ty + 2) * 2 * RW;           // [(ty+1)][2][RW]: Hz, Hx at plane k

  // XCD-aware tile order: consecutive workgroup ids are dealt round-robin to
  // the 8 XCDs, so give each XCD a contiguous run of tiles (neighbouring
  // y-tiles of one z-chunk share halo rows in that XCD's L2).
  const int per_xcd = gridDim.x >> 3;
  const int t = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (t >= a.ntiles) return;
  const int ytile = t % a.ny_tiles;
  const int chunk = t / a.ny_tiles;

  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int j0 = ytile * a.ty;
  const int j = j0 - 1 + w;          // w = 0: halo row j0-1
  const bool halo = (w == 0);
  const bool row_ok = (j >= 0) && (j < a.ny);
  const int k0 = chunk * a.kz;
  const int k1 = min(a.nz, k0 + a.kz);
  const int kstart = k0 > 0 ? k0 - 1 : 0;
  const int x0 = lane * V;
  const bool lane_ok = x0 < a.nx;
  const int nx = a.nx, ny = a.ny, nz = a.nz, px = a.px;
  const size_t plane = (size_t)ny * px;
  const C idx_ = a.inv_d[0], idy = a.inv_d[1], idz = a.inv_d[2];

  bool xin[V];
#pragma unroll
  for (int e = 0; e < V; ++e) xin[e] = (x0 + e) < nx;

  // x-slab membership per element
  const int Lx = a.L[0], Ly = a.L[1], Lz = a.L[2];
  bool inx[V];
  int sx[V];
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const int i = x0 + e;
    inx[e] = xin[e] && (i < Lx || i >= nx - Lx);
    sx[e] = i < Lx ? i : i - nx + 2 * Lx;
  }
  const bool iny = row_ok && (j < Ly || j >= ny - Ly);
  const int sy = j < Ly ? j : j - ny + 2 * Ly;

  int segx[V];
#pragma unroll
  for (int e = 0; e < V; ++e) segx[e] = xin[e] ? a.segx[x0 + e] : 0;
  const int segy = row_ok ? a.segy[j] * a.nsx : 0;

  const bool ld_ok = row_ok && lane_ok;
  C ec[3][V];  // E^n(k)
  {
    const size_t off = (size_t)kstart * plane + (size_t)max(j, 0) * px + x0;
#pragma unroll
    for (int c = 0; c < 3; ++c) load_row<T, C, V>(a.e_in[c] + off, ld_ok, ec[c], a.dec[c]);
  }
  C hxp[V], hyp[V];  // H^{n+1/2}(k-1), own row
#pragma unroll
  for (int e = 0; e < V; ++e) { hxp[e] = C(0); hyp[e] = C(0); }

  for (int k = kstart; k < k1; ++k) {
    const bool active = k >= k0;
    const size_t off = (size_t)k * plane + (size_t)max(j, 0) * px + x0;
    C en[3][V];  // E^n(k+1)
    const bool nx_ok = ld_ok && (k + 1 < nz);
#pragma unroll
    for (int c = 0; c < 3; ++c) load_row<T, C, V>(a.e_in[c] + off + plane, nx_ok, en[c], a.dec[c]);
    C ho[3][V];  // H^{n-1/2}(k)
    load_row<T, C, V>(a.h_in[0] + off, ld_ok, ho[0], a.dec[3]);
    load_row<T, C, V>(a.h_in[1] + off, ld_ok && !halo, ho[1], a.dec[4]);
    load_row<T, C, V>(a.h_in[2] + off, ld_ok, ho[2], a.dec[5]);

    if (halo) {
      // the row above the tile: Ez, Ex at plane k
      const int jt = j0 + a.ty;
      const bool ok = lane_ok && jt < ny;
      const size_t offt = (size_t)k * plane + (size_t)min(jt, ny - 1) * px + x0;
      C tz[V], tx[V];
      load_row<T, C, V>(a.e_in[2] + offt, ok, tz, a.dec[2]);
      load_row<T, C, V>(a.e_in[0] + offt, ok, tx, a.dec[0]);
      C* r = ldsE + (a.ty + 1) * 2 * RW;
#pragma unroll
      for (int e = 0; e < V; ++e) { r[x0 + e] = tz[e]; r[RW + x0 + e] = tx[e]; }
    }
    {
      C* r = ldsE + w * 2 * RW;
#pragma unroll
      for (int e = 0; e < V; ++e) { r[x0 + e] = ec[2][e]; r[RW + x0 + e] = ec[0][e]; }
    }
    __syncthreads();
    C ezu[V], exu[V];  // Ez, Ex at row j+1
    {
      const C* r = ldsE + (w + 1) * 2 * RW;
#pragma unroll
      for (int e = 0; e < V; ++e) { ezu[e] = r[x0 + e]; exu[e] = r[RW + x0 + e]; }
    }

    // ---------------- H half step at plane k ----------------
    const bool inz = (k < Lz || k >= nz - Lz);
    const bool inz_r = inz && row_ok;
    const int sz = k < Lz ? k : k - nz + 2 * Lz;
    const bool upd_psi = active && !halo && row_ok;
    const C ez_r = shfl_down1(ec[2][0], lane);
    const C ey_r = shfl_down1(ec[1][0], lane);
    C hx[V], hy[V], hz[V];
    {
      // scalar CPML coefficients for the row (y) and plane (z), H side
      C byh = 1, ayh = 0, kyh = 1, bzh = 1, azh = 0, kzh = 1;
      if (iny) { byh = a.pb[1][1][j]; ayh = a.pa[1][1][j]; kyh = a.pk[1][1][j]; }
      if (inz) { bzh = a.pb[1][2][k]; azh = a.pa[1][2][k]; kzh = a.pk[1][2][k]; }
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const int i = x0 + e;
        const C ezn = (e < V - 1) ? ec[2][e + 1] : ez_r;
        const C eyn = (e < V - 1) ? ec[1][e + 1] : ey_r;
        C dEz_dy = (ezu[e] - ec[2][e]) * idy;
        C dEy_dz = (en[1][e] - ec[1][e]) * idz;
        C dEx_dz = (en[0][e] - ec[0][e]) * idz;
        C dEz_dx = (ezn - ec[2][e]) * idx_;
        C dEy_dx = (eyn - ec[1][e]) * idx_;
        C dEx_dy = (exu[e] - ec[0][e]) * idy;
        if (iny && xin[e]) {
          const size_t q = ((size_t)k * (2 * Ly) + sy) * px + i;
          C p1 = byh * a.psi_h_in[PHXY][q] + ayh * dEz_dy;
          C p2 = byh * a.psi_h_in[PHZY][q] + ayh * dEx_dy;
          if (upd_psi) { a.psi_h_out[PHXY][q] = p1; a.psi_h_out[PHZY][q] = p2; }
          dEz_dy = kyh * dEz_dy + p1;
          dEx_dy = kyh * dEx_dy + p2;
        }
        if (inz_r && xin[e]) {
          const size_t q = ((size_t)sz * ny + j) * px + i;
          C p1 = bzh * a.psi_h_in[PHXZ][q] + azh * dEy_dz;
          C p2 = bzh * a.psi_h_in[PHYZ][q] + azh * dEx_dz;
          if (upd_psi) { a.psi_h_out[PHXZ][q] = p1; a.psi_h_out[PHYZ][q] = p2; }
          dEy_dz = kzh * dEy_dz + p1;
          dEx_dz = kzh * dEx_dz + p2;
        }
        if (inx[e] && row_ok) {
          const size_t q = ((size_t)k * ny + j) * (2 * Lx) + sx[e];
          const C bxh = a.pb[1][0][i], axh = a.pa[1][0][i], kxh = a.pk[1][0][i];
          C p1 = bxh * a.psi_h_in[PHYX][q] + axh * dEz_dx;
          C p2 = bxh * a.psi_h_in[PHZX][q] + axh * dEy_dx;
          if (upd_psi) { a.psi_h_out[PHYX][q] = p1; a.psi_h_out[PHZX][q] = p2; }
          dEz_dx = kxh * dEz_dx + p1;
          dEy_dx = kxh * dEy_dx + p2;
        }
        const bool ok = row_ok && xin[e];
        hx[e] = ok ? to_storage<T, C>(ho[0][e] - a.dt_mu * (dEz_dy - dEy_dz), a.enc[3], a.dec[3]) : C(0);
        hy[e] = ok ? to_storage<T, C>(ho[1][e] - a.dt_mu * (dEx_dz - dEz_dx), a.enc[4], a.dec[4]) : C(0);
        hz[e] = ok ? to_storage<T, C>(ho[2][e] - a.dt_mu * (dEy_dx - dEx_dy), a.enc[5], a.dec[5]) : C(0);
      }
    }
    {
      C* r = ldsH + w * 2 * RW;
#pragma unroll
      for (int e = 0; e < V; ++e) { r[x0 + e] = hz[e]; r[RW + x0 + e] = hx[e]; }
    }
    __syncthreads();

    // ---------------- E half step at plane k (own rows) ----------------
    if (!halo && active && row_ok && lane_ok) {
      C hzd[V], hxd[V];  // Hz, Hx at row j-1
      {
        const C* r = ldsH + (w - 1) * 2 * RW;
#pragma unroll
        for (int e = 0; e < V; ++e) { hzd[e] = r[x0 + e]; hxd[e] = r[RW + x0 + e]; }
      }
      const C hy_l = shfl_up1(hy[V - 1], lane);
      const C hz_l = shfl_up1(hz[V - 1], lane);
      C bye = 1, aye = 0, kye = 1, bze = 1, aze = 0, kze = 1;
      if (iny) { bye = a.pb[0][1][j]; aye = a.pa[0][1][j]; kye = a.pk[0][1][j]; }
      if (inz) { bze = a.pb[0][2][k]; aze = a.pa[0][2][k]; kze = a.pk[0][2][k]; }
      const int segyz = segy + a.segz[k] * a.nsxy;
      const int pl = a.pec_plane[k];
      C exo[V], eyo[V], ezo[V];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const int i = x0 + e;
        const C hyl = (e > 0) ? hy[e - 1] : hy_l;
        const C hzl = (e > 0) ? hz[e - 1] : hz_l;
        C dHz_dy = (hz[e] - hzd[e]) * idy;
        C dHy_dz = (hy[e] - hyp[e]) * idz;
        C dHx_dz = (hx[e] - hxp[e]) * idz;
        C dHz_dx = (hz[e] - hzl) * idx_;
        C dHy_dx = (hy[e] - hyl) * idx_;
        C dHx_dy = (hx[e] - hxd[e]) * idy;
        // wall samples (tangential E on the outer faces) are never updated
        const bool ux = (j > 0) && (k > 0) && xin[e];
        const bool uy = (i > 0) && (k > 0) && xin[e];
        const bool uz = (i > 0) && (j > 0) && xin[e];
        if (iny && xin[e]) {
          const size_t q = ((size_t)k * (2 * Ly) + sy) * px + i;
          if (ux) { C p = bye * a.psi_e[PEXY][q] + aye * dHz_dy; a.psi_e[PEXY][q] = p; dHz_dy = kye * dHz_dy + p; }
          if (uz) { C p = bye * a.psi_e[PEZY][q] + aye * dHx_dy; a.psi_e[PEZY][q] = p; dHx_dy = kye * dHx_dy + p; }
        }
        if (inz && xin[e]) {
          const size_t q = ((size_t)sz * ny + j) * px + i;
          if (ux) { C p = bze * a.psi_e[PEXZ][q] + aze * dHy_dz; a.psi_e[PEXZ][q] = p; dHy_dz = kze * dHy_dz + p; }
          if (uy) { C p = bze * a.psi_e[PEYZ][q] + aze * dHx_dz; a.psi_e[PEYZ][q] = p; dHx_dz = kze * dHx_dz + p; }
        }
        if (inx[e]) {
          const size_t q = ((size_t)k * ny + j) * (2 * Lx) + sx[e];
          const C bxe = a.pb[0][0][i], axe = a.pa[0][0][i], kxe = a.pk[0][0][i];
          if (uy) { C p = bxe * a.psi_e[PEYX][q] + axe * dHz_dx; a.psi_e[PEYX][q] = p; dHz_dx = kxe * dHz_dx + p; }
          if (uz) { C p = bxe * a.psi_e[PEZX][q] + axe * dHy_dx; a.psi_e[PEZX][q] = p; dHy_dx = kxe * dHy_dx + p; }
        }
        const Coef2<C> cc = a.coef[segx[e] + segyz];
        C ca = cc.ca, cb = cc.cb;
        C cax = ca, cbx = cb, cay = ca, cby = cb, caz = ca, cbz = cb;
        if (pl >= 0) {
          const uint8_t m = a.pec_mask[((size_t)pl * ny + j) * px + min(i, px - 1)];
          if (m & 1) { cax = C(0); cbx = C(0); }
          if (m & 2) { cay = C(0); cby = C(0); }
          if (m & 4) { caz = C(0); cbz = C(0); }
        }
        exo[e] = ux ? cax * ec[0][e] + cbx * (dHz_dy - dHy_dz) : ec[0][e];
        eyo[e] = uy ? cay * ec[1][e] + cby * (dHx_dz - dHz_dx) : ec[1][e];
        ezo[e] = uz ? caz * ec[2][e] + cbz * (dHy_dx - dHx_dy) : ec[2][e];
      }
      if (a.rowflag[(size_t)k * ny + j] & 1) {
        const double tn = (double)(a.n + 1) * a.dt;
        for (int s = 0; s < a.nsrc; ++s) {
          const SrcDev sd = a.src[s];
          if (sd.j == j && sd.k == k && sd.i >= x0 && sd.i < x0 + V) {
            const C add = static_cast<C>(sd.amp * waveform(sd, tn));
#pragma unroll
            for (int e = 0; e < V; ++e) {
              if (x0 + e == sd.i) {
                if (sd.comp == 0) exo[e] += add;
                else if (sd.comp == 1) eyo[e] += add;
                else ezo[e] += add;
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
      store_row<T, C, V>(a.e_out[0] + off, exo, a.enc[0]);
      store_row<T, C, V>(a.e_out[1] + off, eyo, a.enc[1]);
      store_row<T, C, V>(a.e_out[2] + off, ezo, a.enc[2]);
      store_row<T, C, V>(a.h_out[0] + off, hx, a.enc[3]);
      store_row<T, C, V>(a.h_out[1] + off, hy, a.enc[4]);
      store_row<T, C, V>(a.h_out[2] + off, hz, a.enc[5]);
      if (a.rowflag[(size_t)k * ny + j] & 2) {
        const int slot = (int)(a.n % a.series_len);
        for (int p = 0; p < a.nprobe; ++p) {
          const int4 pr = a.probe[p];
          if (pr.z == j && pr.w == k && pr.y >= x0 && pr.y < x0 + V) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
              if (x0 + e == pr.y) {
                C v = pr.x == 0 ? exo[e] : pr.x == 1 ? eyo[e] : pr.x == 2 ? ezo[e]
                    : pr.x == 3 ? hx[e] : pr.x == 4 ? hy[e] : hz[e];
                a.series[(size_t)slot * a.nprobe + p] = static_cast<double>(v);
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
      for (int c = 0; c < 3; ++c) ec[c][e] = en[c][e];
    }
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
