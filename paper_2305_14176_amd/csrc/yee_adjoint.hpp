// Device kernels of the discrete adjoint (reverse-mode derivative) of the Yee
// step in yee_kernels.hpp.
//
// Forward step n, written as sub-maps (psi_H, H, psi_E, E, source, objective):
//   psi_H' = b psi_H + a D_f E           H' = H - (dt/mu0) sum_t s_t (kinv_t D_f E + psi_H')
//   psi_E' = b psi_E + a D_b H'          E' = Ca E + Cb sum_t s_t (kinv_t D_b H' + psi_E')
//   E' += source (state independent)     J += sum_p y_p^2 (probe samples of the new state)
// (D_f / D_b: forward / backward differences, s_t = +-1 the sign of curl term t,
// kinv = 1/kappa; CPML recursion after Roden & Gedney 2000).  The reverse step
// applies the transposed sub-maps in the opposite order.  The adjoint of E is
// carried scaled by Cb, u = Cb * E_bar, which turns the transposed E update into
// the same shape as the forward one:
//   1. objective:  u[p] += Cb 2 y_p (E probes), H_bar[p] += 2 y_p (H probes)
//   2. adj_h:      dbar_t = s_t (kinv_t u + a_t (P_t + s_t u))      at E samples
//                  H_bar  += D_b^T dbar_t = sum over the two E samples of each term
//                  P_t    <- b_t (P_t + s_t u)                        (psi_E adjoint)
//   3. adj_e:      gbar_t = -mu s_t (kinv_t H_bar) + a_t (Q_t - mu s_t H_bar) at H samples
//                  grad   += (u/Cb) (dCa/deps E^n + dCb/deps R^n)      (cells of the box)
//                  u      <- Ca u + Cb D_f^T gbar_t
//                  Q_t    <- b_t (Q_t - mu s_t H_bar)                 (psi_H adjoint)
// with mu = dt/mu0 and Cb R^n = E^{n+1} - source - Ca E^n read from the stored
// forward history.  Profiles are those of the sample each term lives on (E
// side for P, H side for Q).  Samples never updated by the forward step (E on
// the outer PEC faces, PEC-masked E) have u = 0.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "yee_kernels.hpp"

namespace yee {

// Unique probed sample of the objective (probes on one sample are summed).
struct InjDev {
  int32_t comp;       // 0..5
  uint32_t off;       // element offset (k * ny + j) * px + i
  int32_t first;      // first probe on this sample
  int32_t i, j, k;
  double w;           // 2 * Cb for E samples (0 if never updated), 2 for H samples
};

template <class T, class C>
struct AdjArgs {
  C* u;                     // Cb * E_bar, component c at u + c * ustride
  C* hb;                    // H_bar, component c at hb + c * ustride
  uint64_t ustride;
  const C* pin;             // psi adjoint (E side in adj_h, H side in adj_e), old
  C* pout;                  // new
  uint32_t psoff[6];        // element offset of the pair array holding each auxiliary (see yee_kernels.hpp)
  const C* prof;            // CPML profiles [side E,H][axis][1 - b | a | 1/kappa][plen]
  int32_t plen;
  const int32_t* seg;       // block index per cell: x [px] | y [ny] | z [nz]
  const Coef2<C>* coef;     // (Ca, Cb) per block
  const double2* dcoef;     // (dCa/deps / Cb, dCb/deps / Cb^2) per block, FP64
  int32_t nsx, nsxy;
  const int32_t* pec_plane;
  const uint8_t* pec_mask;
  const T* hist_n;          // E^n over the box, component c at + c * hstride
  const T* hist_np1;        // E^{n+1} over the box
  uint64_t hstride;
  double* grad;             // [k - k0][j - j0][i - i0], FP64
  int32_t box[6];           // i0, i1, j0, j1, k0, k1
  const SrcDev* src;
  int32_t nsrc;
  int64_t n;                // forward step being reversed
  double dt;
  int32_t nx, ny, nz, px;
  int32_t L[3];
  C inv_d[3];
  C dt_mu;
  // objective seeds folded into the kernels (see adj_inject_kernel)
  const InjDev* inj;        // unique probed samples
  int32_t ninj;
  const int4* probe;        // (comp, i, j, k)
  int32_t nprobe;
  const uint8_t* rowflag;   // [nz][ny], bit 1: a probe in the row
  const double* yrow_h;     // adj_h: probe samples whose H seeds this step adds (or null)
  const double* yrow_e;     // adj_e: probe samples whose E seeds the next reverse step needs (or null)
};

// Threads per workgroup along x, y: two waves of 32 samples of 2 rows each
// (one plane).  At 128^3 the reverse run of 1024 steps took 55.9 ms against
// 61.1 ms with 64 x 4 and 71.0 ms with 64 x 8; 16-wide or one-row shapes
// were slower still.
constexpr int kAdjBX = 32, kAdjBY = 4;

// Seed of probed sample d: w * (sum of the samples of the probes on it).
__device__ __forceinline__ double inj_seed(const InjDev& d, const int4* probe, int nprobe, const double* yrow) {
  double s = 0.0;
  for (int p = d.first; p < nprobe; ++p) {
    const int4 pr = probe[p];
    if (pr.x == d.comp && pr.y == d.i && pr.z == d.j && pr.w == d.k) s += yrow[p];
  }
  return s;
}

// Seeds of the samples of components [c0, c0 + 3) at element offset o.
template <class C>
__device__ __forceinline__ void inj_seeds(const InjDev* inj, int ninj, const int4* probe, int nprobe,
                                          const double* yrow, int c0, uint32_t o, C (&out)[3]) {
  for (int q = 0; q < ninj; ++q) {
    const InjDev d = inj[q];
    if (d.comp >= c0 && d.comp < c0 + 3 && d.off == o)
      out[d.comp - c0] += static_cast<C>(d.w) * static_cast<C>(inj_seed(d, probe, nprobe, yrow));
  }
}

__device__ __forceinline__ bool in_layer(int i, int n, int L) { return i < L || i >= n - L; }
__device__ __forceinline__ int slab(int i, int n, int L) { return i < L ? i : i - n + 2 * L; }

// ---------------------------------------------------------------------------
// 1. Objective: each unique probed sample adds w sum_p y_p[n+1] (w = 2 Cb for
//    E samples, 2 for H samples).  The seeds of a reverse step are folded into
//    the kernels: adj_h adds the H seeds of its own step while it updates
//    H_bar, and adj_e adds the E seeds of the next reverse step as it writes
//    u.  This kernel only seeds u before the first reverse step.
// ---------------------------------------------------------------------------
template <class C>
__global__ void adj_inject_kernel(const InjDev* __restrict__ inj, int ninj, const int4* __restrict__ probe,
                                  int nprobe, const double* __restrict__ yrow, C* u, C* hb,
                                  uint64_t ustride, int comp_end) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= ninj) return;
  const InjDev d = inj[q];
  if (d.comp >= comp_end) return;
  const double s = inj_seed(d, probe, nprobe, yrow);
  C* base = d.comp < 3 ? u + (uint64_t)d.comp * ustride : hb + (uint64_t)(d.comp - 3) * ustride;
  base[d.off] += static_cast<C>(d.w) * static_cast<C>(s);
}

// ---------------------------------------------------------------------------
// 2. Transposed E update, H side: H_bar += D_b^T dbar, psi_E adjoint.
// ---------------------------------------------------------------------------
template <class C>
__global__ void __launch_bounds__(kAdjBX * kAdjBY)
adj_h_kernel(const AdjArgs<C, C> a) {
  const int i = blockIdx.x * kAdjBX + threadIdx.x;
  const int j = blockIdx.y * kAdjBY + threadIdx.y;
  const int k = blockIdx.z;
  const int nx = a.nx, ny = a.ny, nz = a.nz, px = a.px;
  if (i >= nx || j >= ny) return;
  const int Lx = a.L[0], Ly = a.L[1], Lz = a.L[2];
  const uint32_t plane = (uint32_t)ny * px;
  const uint32_t o = (uint32_t)k * plane + (uint32_t)j * px + i;
  const C* U0 = a.u;
  const C* U1 = a.u + a.ustride;
  const C* U2 = a.u + 2 * a.ustride;
  const bool xp = i + 1 < nx, yp = j + 1 < ny, zp = k + 1 < nz;
  const C ux = U0[o], uy = U1[o], uz = U2[o];
  const C ux_y = yp ? U0[o + px] : C(0), uz_y = yp ? U2[o + px] : C(0);
  const C ux_z = zp ? U0[o + plane] : C(0), uy_z = zp ? U1[o + plane] : C(0);
  const C uy_x = xp ? U1[o + 1] : C(0), uz_x = xp ? U2[o + 1] : C(0);
  const C* P = a.pin;
  const C* pr = a.prof;
  const int pl = a.plen;

  // dbar of the y terms (XY: +Ex, ZY: -Ez) at E samples j and j + 1
  C dxy0 = ux, dxy1 = ux_y, dzy0 = -uz, dzy1 = -uz_y;
  if (in_layer(j, ny, Ly)) {
    const uint32_t q = ((uint32_t)k * (2 * Ly) + slab(j, ny, Ly)) * px + i;
    const C kv = pr[5 * pl + j], av = pr[4 * pl + j];
    dxy0 = kv * ux + av * (P[a.psoff[PEXY] + 2 * q + psi_member(PEXY)] + ux);
    dzy0 = -kv * uz + av * (P[a.psoff[PEZY] + 2 * q + psi_member(PEZY)] - uz);
  }
  if (yp && in_layer(j + 1, ny, Ly)) {
    const uint32_t q = ((uint32_t)k * (2 * Ly) + slab(j + 1, ny, Ly)) * px + i;
    const C kv = pr[5 * pl + j + 1], av = pr[4 * pl + j + 1];
    dxy1 = kv * ux_y + av * (P[a.psoff[PEXY] + 2 * q + psi_member(PEXY)] + ux_y);
    dzy1 = -kv * uz_y + av * (P[a.psoff[PEZY] + 2 * q + psi_member(PEZY)] - uz_y);
  }
  // z terms (YZ: +Ey, XZ: -Ex) at k and k + 1
  C dyz0 = uy, dyz1 = uy_z, dxz0 = -ux, dxz1 = -ux_z;
  if (in_layer(k, nz, Lz)) {
    const uint32_t q = ((uint32_t)slab(k, nz, Lz) * ny + j) * px + i;
    const C kv = pr[8 * pl + k], av = pr[7 * pl + k];
    dyz0 = kv * uy + av * (P[a.psoff[PEYZ] + 2 * q + psi_member(PEYZ)] + uy);
    dxz0 = -kv * ux + av * (P[a.psoff[PEXZ] + 2 * q + psi_member(PEXZ)] - ux);
  }
  if (zp && in_layer(k + 1, nz, Lz)) {
    const uint32_t q = ((uint32_t)slab(k + 1, nz, Lz) * ny + j) * px + i;
    const C kv = pr[8 * pl + k + 1], av = pr[7 * pl + k + 1];
    dyz1 = kv * uy_z + av * (P[a.psoff[PEYZ] + 2 * q + psi_member(PEYZ)] + uy_z);
    dxz1 = -kv * ux_z + av * (P[a.psoff[PEXZ] + 2 * q + psi_member(PEXZ)] - ux_z);
  }
  // x terms (ZX: +Ez, YX: -Ey) at i and i + 1
  C dzx0 = uz, dzx1 = uz_x, dyx0 = -uy, dyx1 = -uy_x;
  const uint32_t qx = ((uint32_t)k * ny + j) * (2 * Lx);
  if (in_layer(i, nx, Lx)) {
    const uint32_t q = qx + slab(i, nx, Lx);
    const C kv = pr[2 * pl + i], av = pr[1 * pl + i];
    dzx0 = kv * uz + av * (P[a.psoff[PEZX] + 2 * q + psi_member(PEZX)] + uz);
    dyx0 = -kv * uy + av * (P[a.psoff[PEYX] + 2 * q + psi_member(PEYX)] - uy);
  }
  if (xp && in_layer(i + 1, nx, Lx)) {
    const uint32_t q = qx + slab(i + 1, nx, Lx);
    const C kv = pr[2 * pl + i + 1], av = pr[1 * pl + i + 1];
    dzx1 = kv * uz_x + av * (P[a.psoff[PEZX] + 2 * q + psi_member(PEZX)] + uz_x);
    dyx1 = -kv * uy_x + av * (P[a.psoff[PEYX] + 2 * q + psi_member(PEYX)] - uy_x);
  }
  const C idx = a.inv_d[0], idy = a.inv_d[1], idz = a.inv_d[2];
  C* H0 = a.hb;
  C* H1 = a.hb + a.ustride;
  C* H2 = a.hb + 2 * a.ustride;
  C sd[3] = {C(0), C(0), C(0)};   // objective seeds of this step's H samples here
  if (a.yrow_h && (a.rowflag[(uint32_t)k * ny + j] & 2))
    inj_seeds<C>(a.inj, a.ninj, a.probe, a.nprobe, a.yrow_h, 3, o, sd);
  H0[o] = (H0[o] + sd[0]) + ((dzy0 - dzy1) * idy + (dyz0 - dyz1) * idz);
  H1[o] = (H1[o] + sd[1]) + ((dxz0 - dxz1) * idz + (dzx0 - dzx1) * idx);
  H2[o] = (H2[o] + sd[2]) + ((dxy0 - dxy1) * idy + (dyx0 - dyx1) * idx);

  // psi_E adjoint of the own samples: P <- b (P + s u)
  if (in_layer(j, ny, Ly)) {
    const uint32_t q = ((uint32_t)k * (2 * Ly) + slab(j, ny, Ly)) * px + i;
    const C ob = pr[3 * pl + j];
    { const C t = P[a.psoff[PEXY] + 2 * q + psi_member(PEXY)] + ux; a.pout[a.psoff[PEXY] + 2 * q + psi_member(PEXY)] = t - ob * t; }
    { const C t = P[a.psoff[PEZY] + 2 * q + psi_member(PEZY)] - uz; a.pout[a.psoff[PEZY] + 2 * q + psi_member(PEZY)] = t - ob * t; }
  }
  if (in_layer(k, nz, Lz)) {
    const uint32_t q = ((uint32_t)slab(k, nz, Lz) * ny + j) * px + i;
    const C ob = pr[6 * pl + k];
    { const C t = P[a.psoff[PEYZ] + 2 * q + psi_member(PEYZ)] + uy; a.pout[a.psoff[PEYZ] + 2 * q + psi_member(PEYZ)] = t - ob * t; }
    { const C t = P[a.psoff[PEXZ] + 2 * q + psi_member(PEXZ)] - ux; a.pout[a.psoff[PEXZ] + 2 * q + psi_member(PEXZ)] = t - ob * t; }
  }
  if (in_layer(i, nx, Lx)) {
    const uint32_t q = qx + slab(i, nx, Lx);
    const C ob = pr[0 * pl + i];
    { const C t = P[a.psoff[PEZX] + 2 * q + psi_member(PEZX)] + uz; a.pout[a.psoff[PEZX] + 2 * q + psi_member(PEZX)] = t - ob * t; }
    { const C t = P[a.psoff[PEYX] + 2 * q + psi_member(PEYX)] - uy; a.pout[a.psoff[PEYX] + 2 * q + psi_member(PEYX)] = t - ob * t; }
  }
}

// ---------------------------------------------------------------------------
// 3. Transposed H update, E side: u <- Ca u + Cb D_f^T gbar, psi_H adjoint,
//    and the FP64 gradient of the box cells.
// ---------------------------------------------------------------------------
template <class T, class C>
__global__ void __launch_bounds__(kAdjBX * kAdjBY)
adj_e_kernel(const AdjArgs<T, C> a) {
  const int i = blockIdx.x * kAdjBX + threadIdx.x;
  const int j = blockIdx.y * kAdjBY + threadIdx.y;
  const int k = blockIdx.z;
  const int nx = a.nx, ny = a.ny, nz = a.nz, px = a.px;
  if (i >= nx || j >= ny) return;
  const int Lx = a.L[0], Ly = a.L[1], Lz = a.L[2];
  const uint32_t plane = (uint32_t)ny * px;
  const uint32_t o = (uint32_t)k * plane + (uint32_t)j * px + i;
  const C* H0 = a.hb;
  const C* H1 = a.hb + a.ustride;
  const C* H2 = a.hb + 2 * a.ustride;
  const bool xm = i > 0, ym = j > 0, zm = k > 0;
  const C hx = H0[o], hy = H1[o], hz = H2[o];
  const C hx_y = ym ? H0[o - px] : C(0), hz_y = ym ? H2[o - px] : C(0);
  const C hx_z = zm ? H0[o - plane] : C(0), hy_z = zm ? H1[o - plane] : C(0);
  const C hy_x = xm ? H1[o - 1] : C(0), hz_x = xm ? H2[o - 1] : C(0);
  const C mu = a.dt_mu;
  const C* Q = a.pin;
  const C* pr = a.prof;
  const int pl = a.plen;

  // gbar of the y terms (XY: +Hx, ZY: -Hz) at H samples j - 1 and j
  C gxy1 = -mu * hx, gxy0 = -mu * hx_y, gzy1 = mu * hz, gzy0 = mu * hz_y;
  if (in_layer(j, ny, Ly)) {
    const uint32_t q = ((uint32_t)k * (2 * Ly) + slab(j, ny, Ly)) * px + i;
    const C kv = pr[14 * pl + j], av = pr[13 * pl + j];
    gxy1 = -mu * kv * hx + av * (Q[a.psoff[PHXY] + 2 * q + psi_member(PHXY)] - mu * hx);
    gzy1 = mu * kv * hz + av * (Q[a.psoff[PHZY] + 2 * q + psi_member(PHZY)] + mu * hz);
  }
  if (ym && in_layer(j - 1, ny, Ly)) {
    const uint32_t q = ((uint32_t)k * (2 * Ly) + slab(j - 1, ny, Ly)) * px + i;
    const C kv = pr[14 * pl + j - 1], av = pr[13 * pl + j - 1];
    gxy0 = -mu * kv * hx_y + av * (Q[a.psoff[PHXY] + 2 * q + psi_member(PHXY)] - mu * hx_y);
    gzy0 = mu * kv * hz_y + av * (Q[a.psoff[PHZY] + 2 * q + psi_member(PHZY)] + mu * hz_y);
  }
  // z terms (YZ: +Hy, XZ: -Hx) at k - 1 and k
  C gyz1 = -mu * hy, gyz0 = -mu * hy_z, gxz1 = mu * hx, gxz0 = mu * hx_z;
  if (in_layer(k, nz, Lz)) {
    const uint32_t q = ((uint32_t)slab(k, nz, Lz) * ny + j) * px + i;
    const C kv = pr[17 * pl + k], av = pr[16 * pl + k];
    gyz1 = -mu * kv * hy + av * (Q[a.psoff[PHYZ] + 2 * q + psi_member(PHYZ)] - mu * hy);
    gxz1 = mu * kv * hx + av * (Q[a.psoff[PHXZ] + 2 * q + psi_member(PHXZ)] + mu * hx);
  }
  if (zm && in_layer(k - 1, nz, Lz)) {
    const uint32_t q = ((uint32_t)slab(k - 1, nz, Lz) * ny + j) * px + i;
    const C kv = pr[17 * pl + k - 1], av = pr[16 * pl + k - 1];
    gyz0 = -mu * kv * hy_z + av * (Q[a.psoff[PHYZ] + 2 * q + psi_member(PHYZ)] - mu * hy_z);
    gxz0 = mu * kv * hx_z + av * (Q[a.psoff[PHXZ] + 2 * q + psi_member(PHXZ)] + mu * hx_z);
  }
  // x terms (ZX: +Hz, YX: -Hy) at i - 1 and i
  C gzx1 = -mu * hz, gzx0 = -mu * hz_x, gyx1 = mu * hy, gyx0 = mu * hy_x;
  const uint32_t qx = ((uint32_t)k * ny + j) * (2 * Lx);
  if (in_layer(i, nx, Lx)) {
    const uint32_t q = qx + slab(i, nx, Lx);
    const C kv = pr[11 * pl + i], av = pr[10 * pl + i];
    gzx1 = -mu * kv * hz + av * (Q[a.psoff[PHZX] + 2 * q + psi_member(PHZX)] - mu * hz);
    gyx1 = mu * kv * hy + av * (Q[a.psoff[PHYX] + 2 * q + psi_member(PHYX)] + mu * hy);
  }
  if (xm && in_layer(i - 1, nx, Lx)) {
    const uint32_t q = qx + slab(i - 1, nx, Lx);
    const C kv = pr[11 * pl + i - 1], av = pr[10 * pl + i - 1];
    gzx0 = -mu * kv * hz_x + av * (Q[a.psoff[PHZX] + 2 * q + psi_member(PHZX)] - mu * hz_x);
    gyx0 = mu * kv * hy_x + av * (Q[a.psoff[PHYX] + 2 * q + psi_member(PHYX)] + mu * hy_x);
  }
  const C idx = a.inv_d[0], idy = a.inv_d[1], idz = a.inv_d[2];
  // D_f^T: the E sample m collects gbar[m - 1] - gbar[m]
  const C gx = (gzy0 - gzy1) * idy + (gyz0 - gyz1) * idz;
  const C gy = (gxz0 - gxz1) * idz + (gzx0 - gzx1) * idx;
  const C gz = (gyx0 - gyx1) * idx + (gxy0 - gxy1) * idy;

  // coefficients of the own E samples (PEC mask and outer faces: never updated)
  const int blk = a.seg[i] + a.seg[px + j] * a.nsx + a.seg[px + ny + k] * a.nsxy;
  const Coef2<C> cf = a.coef[blk];
  const int pln = a.pec_plane[k];
  const uint32_t m = pln >= 0 ? a.pec_mask[((uint32_t)pln * ny + j) * px + i] : 0u;
  const bool ux_ok = ym && zm && !(m & 1);
  const bool uy_ok = xm && zm && !(m & 2);
  const bool uz_ok = xm && ym && !(m & 4);
  C* U0 = a.u;
  C* U1 = a.u + a.ustride;
  C* U2 = a.u + 2 * a.ustride;
  const C ux = U0[o], uy = U1[o], uz = U2[o];

  // gradient of the box cells, from u before its update
  if (i >= a.box[0] && i < a.box[1] && j >= a.box[2] && j < a.box[3] && k >= a.box[4] && k < a.box[5]) {
    const int bx = a.box[1] - a.box[0], by = a.box[3] - a.box[2];
    const uint32_t h = ((uint32_t)(k - a.box[4]) * by + (j - a.box[2])) * bx + (i - a.box[0]);
    const double2 g = a.dcoef[blk];
    const double ca = static_cast<double>(cf.ca);
    double src[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < a.nsrc; ++s) {
      const SrcDev sd = a.src[s];
      if (sd.i == i && sd.j == j && sd.k == k)
        src[sd.comp] += static_cast<double>(static_cast<C>(sd.amp * waveform(sd, (double)(a.n + 1) * a.dt)));
    }
    double acc = 0.0;
    const bool ok[3] = {ux_ok, uy_ok, uz_ok};
    const C uu[3] = {ux, uy, uz};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (!ok[c]) continue;
      const double en = static_cast<double>(a.hist_n[c * a.hstride + h]);
      const double e1 = static_cast<double>(a.hist_np1[c * a.hstride + h]) - src[c];
      acc += static_cast<double>(uu[c]) * (g.x * en + g.y * (e1 - ca * en));
    }
    a.grad[h] += acc;
  }

  C sd[3] = {C(0), C(0), C(0)};   // objective seeds of the next reverse step's E samples here
  if (a.yrow_e && (a.rowflag[(uint32_t)k * ny + j] & 2))
    inj_seeds<C>(a.inj, a.ninj, a.probe, a.nprobe, a.yrow_e, 0, o, sd);
  U0[o] = (ux_ok ? cf.ca * ux + cf.cb * gx : C(0)) + sd[0];
  U1[o] = (uy_ok ? cf.ca * uy + cf.cb * gy : C(0)) + sd[1];
  U2[o] = (uz_ok ? cf.ca * uz + cf.cb * gz : C(0)) + sd[2];

  // psi_H adjoint of the own samples: Q <- b (Q - mu s H_bar)
  if (in_layer(j, ny, Ly)) {
    const uint32_t q = ((uint32_t)k * (2 * Ly) + slab(j, ny, Ly)) * px + i;
    const C ob = pr[12 * pl + j];
    { const C t = Q[a.psoff[PHXY] + 2 * q + psi_member(PHXY)] - mu * hx; a.pout[a.psoff[PHXY] + 2 * q + psi_member(PHXY)] = t - ob * t; }
    { const C t = Q[a.psoff[PHZY] + 2 * q + psi_member(PHZY)] + mu * hz; a.pout[a.psoff[PHZY] + 2 * q + psi_member(PHZY)] = t - ob * t; }
  }
  if (in_layer(k, nz, Lz)) {
    const uint32_t q = ((uint32_t)slab(k, nz, Lz) * ny + j) * px + i;
    const C ob = pr[15 * pl + k];
    { const C t = Q[a.psoff[PHYZ] + 2 * q + psi_member(PHYZ)] - mu * hy; a.pout[a.psoff[PHYZ] + 2 * q + psi_member(PHYZ)] = t - ob * t; }
    { const C t = Q[a.psoff[PHXZ] + 2 * q + psi_member(PHXZ)] + mu * hx; a.pout[a.psoff[PHXZ] + 2 * q + psi_member(PHXZ)] = t - ob * t; }
  }
  if (in_layer(i, nx, Lx)) {
    const uint32_t q = qx + slab(i, nx, Lx);
    const C ob = pr[9 * pl + i];
    { const C t = Q[a.psoff[PHZX] + 2 * q + psi_member(PHZX)] - mu * hz; a.pout[a.psoff[PHZX] + 2 * q + psi_member(PHZX)] = t - ob * t; }
    { const C t = Q[a.psoff[PHYX] + 2 * q + psi_member(PHYX)] + mu * hy; a.pout[a.psoff[PHYX] + 2 * q + psi_member(PHYX)] = t - ob * t; }
  }
}

// ---------------------------------------------------------------------------
// Forward history: E of the box cells into one slot [3][bz][by][bx].
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(kAdjBX * kAdjBY)
adj_store_kernel(const T* __restrict__ fields, uint64_t cstride, int ny, int px, int4 lo, int bx, int by,
                 T* __restrict__ slot, uint64_t hstride) {
  const int di = blockIdx.x * kAdjBX + threadIdx.x;
  const int dj = blockIdx.y * kAdjBY + threadIdx.y;
  const int dk = blockIdx.z;
  if (di >= bx || dj >= by) return;
  const uint64_t o = ((uint64_t)(lo.z + dk) * ny + (lo.y + dj)) * px + (lo.x + di);
  const uint64_t h = ((uint64_t)dk * by + dj) * bx + di;
#pragma unroll
  for (int c = 0; c < 3; ++c) slot[c * hstride + h] = fields[c * cstride + o];
}

// Probe ring -> full probe history: y_p[s] for s = s0 + 1 .. s0 + count.
__global__ void adj_gather_kernel(const double* __restrict__ ring, int nprobe, int series_len, int64_t s0,
                                  int count, double* __restrict__ hist) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count * nprobe) return;
  const int64_t s = s0 + 1 + t / nprobe;
  const int p = t % nprobe;
  hist[(size_t)(s - 1) * nprobe + p] = ring[(size_t)((s - 1) % series_len) * nprobe + p];
}

// J = sum of squares of the probe history, one workgroup, fixed order (FP64).
__global__ void __launch_bounds__(256) adj_objective_kernel(const double* __restrict__ hist, int64_t count,
                                                            double* __restrict__ out) {
  __shared__ double part[256];
  double s = 0.0;
  for (int64_t q = threadIdx.x; q < count; q += 256) s += hist[q] * hist[q];
  part[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = part[0];
}

}  // namespace yee
