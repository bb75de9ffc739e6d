// Two leapfrog steps per sweep of the grid (temporal blocking) for gfx950.
//
// The operation is the step of yee_kernels.hpp applied twice (Yee 1966
// staggering and leapfrog; Taflove & Hagness ch. 3 lossy Ca/Cb update;
// Roden & Gedney 2000 CPML recursion).  One sweep reads E^n, H^{n-1/2} and
// the CPML auxiliaries once from HBM and writes E^{n+2}, H^{n+3/2} and the
// auxiliaries once: half the bytes per cell-update of a single-step sweep.
// Every sample is computed with the per-sample arithmetic of yee_kernels.hpp
// (fdiff, cpml_term, h_new, e_new, in the same order), so a two-step sweep is
// bitwise equal to two single steps.
//
// Tile.  A workgroup owns the y-rows [j0, j0+ty) over the full x extent (one
// wave per row, V consecutive x samples per lane, nx <= 64 V) and the z-planes
// [k0, k1), and marches upward in z.  The first step is also computed on the
// halo the second step needs: rows j0-2 .. j0+ty (wave w holds row j0-2+w, so
// the workgroup has ty+3 waves; the row j0+ty+1 above is loaded by the top
// wave) and planes k0-2 .. k1.  At plane p the march runs four stages,
// separated by workgroup barriers:
//   A  H^{n+1/2}(p)   from E^n(p), E^n(p+1), H^{n-1/2}(p)          rows j0-2 .. j0+ty
//   B  E^{n+1}(p)     from E^n(p), H^{n+1/2}(p), H^{n+1/2}(p-1)     rows j0-1 .. j0+ty
//   C  H^{n+3/2}(p-1) from E^{n+1}(p-1), E^{n+1}(p), H^{n+1/2}(p-1) rows j0-1 .. j0+ty-1
//   D  E^{n+2}(p-1)   from E^{n+1}(p-1), H^{n+3/2}(p-1), H^{n+3/2}(p-2)  rows j0 .. j0+ty-1
// y neighbours come from LDS rows, x neighbours from the adjacent lane (DPP
// wave shifts; the shifted-in value beyond either end of the row is 0, the
// PEC wall or the zero sample beyond nx), z neighbours from registers.
// Everything the tile reads is old state (E^n, H^{n-1/2}, auxiliaries before
// the sweep) and everything it writes is new state in the other buffers, so
// tiles that recompute a neighbour's halo never see its results.
//
// CPML auxiliaries.  Each is advanced at both steps; between them the y- and
// z-layer ones stay in registers, the x-layer ones in LDS (a few samples per
// row).  E- and H-side auxiliaries are both ping-ponged here.
#pragma once

#include "yee_kernels.hpp"

namespace yee {


// lane i gets lane i+1's value (0 into lane 63)
__device__ __forceinline__ float from_next_lane(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x130, 0xF, 0xF, true));
}
// lane i gets lane i-1's value (0 into lane 0)
__device__ __forceinline__ float from_prev_lane(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x138, 0xF, 0xF, true));
}

// E component `c` (0..2) of a lane's three samples arrays, without dynamic
// register indexing
template <class C, int V>
__device__ __forceinline__ void add_to_comp(C (&f)[3][V], int c, int e, C v) {
  // selects of values (a branch per component lets the compiler merge the
  // stores through a pointer, which moves the arrays to scratch memory)
  f[0][e] = c == 0 ? f[0][e] + v : f[0][e];
  f[1][e] = c == 1 ? f[1][e] + v : f[1][e];
  f[2][e] = c == 2 ? f[2][e] + v : f[2][e];
}
// identity lane move the optimizer cannot see through: a select among its
// results stays a select of register values (a select among array elements
// would be turned into a load through a selected pointer, which moves the
// arrays to scratch memory)
__device__ __forceinline__ float opaque(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xE4, 0xF, 0xF, false));
}
template <class C, int V>
__device__ __forceinline__ C pick_comp(const C (&ef)[3][V], const C (&hf)[3][V], int c, int e) {
  C v = opaque(hf[2][e]);
  v = c == 4 ? opaque(hf[1][e]) : v;
  v = c == 3 ? opaque(hf[0][e]) : v;
  v = c == 2 ? opaque(ef[2][e]) : v;
  v = c == 1 ? opaque(ef[1][e]) : v;
  v = c == 0 ? opaque(ef[0][e]) : v;
  return v;
}


// A pair of FP32 auxiliaries as one 8-byte buffer access, built from and split
// into register values directly (a bit cast through a two-member struct
// makes the compiler stage the arrays it came from in scratch memory).
__device__ __forceinline__ void ld_pair_f32(rsrc_t r, uint32_t vo, uint32_t so, float& a0, float& a1) {
  const u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0);
  // (elements copied out first: a bit cast applied to a vector element
  // expression reads element 0 whatever the element)
  const unsigned int v0 = v.x, v1 = v.y;
  a0 = __builtin_bit_cast(float, v0);
  a1 = __builtin_bit_cast(float, v1);
}
__device__ __forceinline__ void st_pair_f32(rsrc_t r, uint32_t vo, uint32_t so, float a0, float a1, bool nt) {
  // (opaque: otherwise the two values are gathered through scratch memory)
  u32x2 v;
  v.x = __builtin_bit_cast(unsigned int, opaque(a0));
  v.y = __builtin_bit_cast(unsigned int, opaque(a1));
  if (nt)
    __builtin_amdgcn_raw_buffer_store_b64(v, r, vo, so, 2);
  else
    __builtin_amdgcn_raw_buffer_store_b64(v, r, vo, so, 0);
}

// LDS bytes of one two-step workgroup: ty rows per tile, V samples per lane,
// wpr waves per row, kz planes per chunk (rows of RL = 64 V wpr samples).
//   X[2]  [ty+4][2][64V]   E rows (Ez, Ex) by plane parity: E^n(p) for stages A
//                          and B, then E^{n+1}(p) from B (read by C and D)
//   HA[2] [ty+3][3][64V]   H^{n+1/2}(p) (Hx, Hy, Hz) by plane parity (B: row j-1
//                          and plane p-1; C: the row's own values)
//   Hb    [ty+4][2][64V]   H^{n+3/2}(p-1) rows (Hz, Hx) for stage D
//   seam  [5][ty+4]        two waves per row: the values x neighbours take from
//                          the row's other wave that no row above holds (Ey of
//                          E^n and E^{n+1} by parity, Hy of H^{n+3/2})
//   PX[2] [ty+3][4][2Lx]   x-layer auxiliaries after the first step (H: YX, ZX;
//                          E: YX, ZX) by plane parity
//   HO    [ty+3][8][64V]   y- and z-layer auxiliaries after the first step (H: XY,
//                          ZY, XZ, YZ; E: XY, ZY, XZ, YZ); each row's slots are
//                          read and rewritten by that row's waves only
//   src   [2][kMaxSources] waveform values of the two steps
//   tzp   [6][kz+3]        z profiles of the tile's planes (E side 1-b, a, 1/kappa; H side)
//   txp   [6][64V]         x profiles
//   typ   [6][ty+3]        y profiles of the tile's rows
//   int32 tzs, tzl [kz+3]  z block offset, PEC plane index; uint8 tfl [ty+3][kz+3] row flags
__host__ __device__ inline size_t tb_lds_bytes_for(int ty, int V, int wpr, int kz, int Lx) {
  const size_t rl = (size_t)kWave * V * wpr;
  const size_t nr = (size_t)ty + 4, nw = (size_t)ty + 3, npl = (size_t)kz + 3;
  size_t b = (2 * nr * 2 * rl + 2 * nw * 3 * rl + nr * 2 * rl + 5 * nr + 2 * nw * 4 * 2 * (size_t)Lx + nw * 8 * rl +
              2 * kMaxSources + 6 * npl + 6 * rl + 6 * nw) * 4;
  b += 2 * npl * 4 + nw * npl;
  return (b + 15) & ~size_t(15);
}

// Wave roles of the two-step march (a type): the bottom halo row j0-2 (stage A
// only), the rows j0-1 .. j0+ty-1 (all stages the row takes part in), the top
// halo row j0+ty (stages A and B, and the loads of the row above it).
template <int N>
struct TbRole {
  static constexpr int value = N;
};

template <class T, class C, int V, int WPR, bool NT>
__device__ __forceinline__ void tb_tile(const StepArgs<T, C>& a, const int ytile, const int k0, const int k1,
                                        unsigned char* smem) {
  static_assert(sizeof(C) == 4, "two-step sweeps compute in FP32");
  constexpr int RL = kWave * V * WPR;     // samples per row (WPR waves of 64 V)
  const int ty = a.ty;
  constexpr bool nt = NT;   // stores streamed past the last-level cache
  const int NR = ty + 4, NW = ty + 3;
  const int nx = a.nx, ny = a.ny, nz = a.nz, px = a.px;
  const int Lx = a.L[0], Ly = a.L[1], Lz = a.L[2];
  const int j0 = ytile * ty;
  const int pbeg = k0 >= 2 ? k0 - 2 : 0;
  const int npl = a.kz + 3;               // table stride (planes of the longest chunk)
  const int nq = k1 - pbeg + 1;           // planes pbeg .. k1 this tile visits
  C* X0 = reinterpret_cast<C*>(smem);
  C* HA0 = X0 + 2 * NR * 2 * RL;
  C* Hb = HA0 + 2 * NW * 3 * RL;
  C* seam = Hb + NR * 2 * RL;            // [5][NR]: Ey^n by parity, Ey^{n+1} by parity, Hy^{n+3/2}
  const int XW = 2 * Lx;
  C* PX = seam + 5 * NR;                 // [2][NW][4][XW]
  C* HO = PX + 2 * NW * 4 * XW;          // [NW][8][RL]
  C* ldsS = HO + NW * 8 * RL;
  C* tzp = ldsS + 2 * kMaxSources;
  C* txp = tzp + 6 * npl;
  C* typ = txp + 6 * RL;
  int32_t* tzs = reinterpret_cast<int32_t*>(typ + 6 * NW);
  int32_t* tzl = tzs + npl;
  uint8_t* tfl = reinterpret_cast<uint8_t*>(tzl + npl);
  const int tid = threadIdx.x, nthr = blockDim.x;

  // ---- per-workgroup tables ----
  if (tid < a.nsrc) {
    const SrcDev sd = a.src[tid];
    ldsS[tid] = static_cast<C>(sd.amp * waveform(sd, (double)(a.n + 1) * a.dt));
    ldsS[kMaxSources + tid] = static_cast<C>(sd.amp * waveform(sd, (double)(a.n + 2) * a.dt));
  }
  for (int q = tid; q < nq; q += nthr) {
    const int k = pbeg + q;
    const bool ok = k < nz;
    const bool inz = ok && (k < Lz || k >= nz - Lz);
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int side = u / 3, qq = u % 3;
      tzp[u * npl + q] = inz ? a.prof[((side * 3 + 2) * 3 + qq) * a.plen + k] : (qq == 2 ? C(1) : C(0));
    }
    tzs[q] = ok ? a.seg[px + ny + k] * a.nsxy : 0;
    tzl[q] = ok ? a.pec_plane[k] : -1;
  }
  for (int q = tid; q < 6 * RL; q += nthr) {
    const int u = q / RL, i = q - u * RL;
    const int side = u / 3, qq = u % 3;
    const bool inx = i < nx && (i < Lx || i >= nx - Lx);
    txp[q] = inx ? a.prof[((side * 3 + 0) * 3 + qq) * a.plen + i] : (qq == 2 ? C(1) : C(0));
  }
  for (int q = tid; q < 6 * NW; q += nthr) {
    const int u = q / NW, rr = q - u * NW;
    const int side = u / 3, qq = u % 3;
    const int jj = j0 - 2 + rr;
    const bool iny = jj >= 0 && jj < ny && (jj < Ly || jj >= ny - Ly);
    typ[q] = iny ? a.prof[((side * 3 + 1) * 3 + qq) * a.plen + jj] : (qq == 2 ? C(1) : C(0));
  }
  for (int q = tid; q < NW * nq; q += nthr) {
    const int rr = q / nq, kk = q - rr * nq;
    const int jj = j0 - 2 + rr, k = pbeg + kk;
    tfl[rr * npl + kk] = (jj >= 0 && jj < ny && k < nz) ? a.rowflag[(uint32_t)k * ny + jj] : 0;
  }
  __syncthreads();

  // ---- wave (uniform) ----
  const int wid = uniform(tid >> 6);
  const int wv = wid / WPR;                            // row of the tile (0: j0-2)
  const int half = wid - wv * WPR;                     // x segment of the row
  const int lane = tid & 63;
  const int j = j0 - 2 + wv;
  const bool rowA = j >= 0 && j < ny;                  // stage A on this row
  const bool rowC = rowA && wv >= 1 && wv <= ty + 1;   // stage C
  const bool rowD = rowA && wv >= 2 && wv <= ty + 1;   // stage D: the tile's own rows
  const int jt = j0 + ty + 1;                          // row above the halo (top wave)
  const int jc = min(max(j, 0), ny - 1);
  const bool iny = rowA && (j < Ly || j >= ny - Ly);
  const int sy = j < Ly ? j : j - ny + 2 * Ly;

  // ---- per-lane offsets (kOut: nothing there) ----
  const int xl = half * kWave * V + lane * V;
  // the seam between the two waves of a row: the last lane of the first wave
  // takes its x+1 neighbours, the first lane of the second its x-1 ones, from LDS
  const bool seam_hi = WPR == 2 && half == 0 && lane == kWave - 1;
  const bool seam_lo = WPR == 2 && half == 1 && lane == 0;
  constexpr int XS = kWave * V;                        // first sample of the second wave
  const bool lane_ok = xl < nx;
  constexpr uint32_t TB = sizeof(T), CB = sizeof(C);
  const uint32_t plane = (uint32_t)ny * (uint32_t)px;
  const uint32_t vrow = (rowA && lane_ok) ? ((uint32_t)jc * (uint32_t)px + (uint32_t)xl) * TB : kOut;
  const uint32_t vxc = (rowA && lane_ok) ? (uint32_t)xl * 2 * CB : kOut;   // y/z-slab pairs
  uint32_t vxs[V], vcf[V];
  int xs_slot[V];   // the sample's place in the x layer, or -1
  bool lane_inx = false;
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const int i = xl + e;
    const bool inx = rowA && i < nx && (i < Lx || i >= nx - Lx);
    lane_inx = lane_inx || inx;
    xs_slot[e] = inx ? (i < Lx ? i : i - nx + 2 * Lx) : -1;
    vxs[e] = inx ? (uint32_t)xs_slot[e] * 2 * CB : kOut;
    vcf[e] = (rowA && i < nx) ? (uint32_t)(a.seg[i] + a.seg[px + jc] * a.nsx) * (uint32_t)sizeof(Coef2<C>) : kOut;
  }
  const uint32_t plane_b = plane * TB;
  const uint32_t cs_b = (uint32_t)(a.cstride * TB);
  const rsrc_t rin = make_rsrc(a.fin, 6 * cs_b);
  const rsrc_t rout = make_rsrc(a.fout, 6 * cs_b);
  // the four auxiliary regions (E and H side, old and new) under one resource
  // based at the lowest of them (the host keeps their span below 2 GiB)
  const char* psb = reinterpret_cast<const char*>(a.psbase);
  auto pof = [&](const C* r) __attribute__((always_inline)) { return (uint32_t)(reinterpret_cast<const char*>(r) - psb); };
  const uint32_t pe_in = pof(a.pse), pe_out = pof(a.pse_out);
  const uint32_t ph_in = pof(a.psh_in), ph_out = pof(a.psh_out);
  const rsrc_t rpsi = make_rsrc(psb, a.psi_span);
  const rsrc_t rcoef = make_rsrc(a.coef, a.coef_bytes);
  const C idx_ = a.inv_d[0], idy = a.inv_d[1], idz = a.inv_d[2];
  const C dtm = a.dt_mu;
  auto yso = [&](int k, int q) __attribute__((always_inline)) { return (a.psoff[q] + ((uint32_t)k * (2 * Ly) + sy) * (uint32_t)px * 2) * CB; };
  auto zso = [&](int k, int q) __attribute__((always_inline)) {
    const int sz = k < Lz ? k : k - nz + 2 * Lz;
    return (a.psoff[q] + ((uint32_t)sz * ny + jc) * (uint32_t)px * 2) * CB;
  };
  auto xso = [&](int k, int q) __attribute__((always_inline)) { return (a.psoff[q] + ((uint32_t)k * ny + jc) * (uint32_t)(2 * Lx) * 2) * CB; };
  auto in_z = [&](int k) __attribute__((always_inline)) { return k < nz && (k < Lz || k >= nz - Lz); };

  auto load_E = [&](uint32_t vo, int k, C (&out)[3][V]) __attribute__((always_inline)) {
    const uint32_t so = (uint32_t)k * plane_b;   // k <= nz: plane nz is the zero plane
    ld_row<T, C, V>(rin, vo, so, out[0], a.dec[0]);
    ld_row<T, C, V>(rin, vo, so + cs_b, out[1], a.dec[1]);
    ld_row<T, C, V>(rin, vo, so + 2 * cs_b, out[2], a.dec[2]);
  };
  auto load_ExEz = [&](uint32_t vo, int k, C (&out)[2][V]) __attribute__((always_inline)) {
    const uint32_t so = (uint32_t)k * plane_b;
    ld_row<T, C, V>(rin, vo, so, out[0], a.dec[0]);
    ld_row<T, C, V>(rin, vo, so + 2 * cs_b, out[1], a.dec[2]);
  };
  auto load_H = [&](int k, C (&out)[3][V]) __attribute__((always_inline)) {
    const uint32_t so = 3 * cs_b + (uint32_t)k * plane_b;
    ld_row<T, C, V>(rin, vrow, so, out[0], a.dec[3]);
    ld_row<T, C, V>(rin, vrow, so + cs_b, out[1], a.dec[4]);
    ld_row<T, C, V>(rin, vrow, so + 2 * cs_b, out[2], a.dec[5]);
  };
  // CPML auxiliary pairs of plane k: y/z slabs (one pair per sample), x slab
  // (exec-masked to the lanes holding layer samples)
  auto ld_pair = [&](uint32_t off, C (&o0)[V], C (&o1)[V]) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < V; ++e) ld_pair_f32(rpsi, vxc + e * 2 * CB, off, o0[e], o1[e]);
  };
  auto st_pair = [&](uint32_t off, const C (&i0)[V], const C (&i1)[V]) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < V; ++e) st_pair_f32(rpsi, vxc + e * 2 * CB, off, i0[e], i1[e], nt);
  };
  auto ld_xpair = [&](uint32_t off, C (&o0)[V], C (&o1)[V]) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < V; ++e) ld_pair_f32(rpsi, vxs[e], off, o0[e], o1[e]);
  };
  auto st_xpair = [&](uint32_t off, const C (&i0)[V], const C (&i1)[V]) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < V; ++e) st_pair_f32(rpsi, vxs[e], off, i0[e], i1[e], nt);
  };
  // auxiliaries of plane k at region base `rb` (H side: (XY, ZY), (XZ, YZ), (YX, ZX))
  struct Aux {
    C y0[V], y1[V], z0[V], z1[V], x0[V], x1[V];
  };
  auto aux_zero = [&](Aux& u) __attribute__((always_inline)) {
#pragma unroll
    for (int e = 0; e < V; ++e) u.y0[e] = u.y1[e] = u.z0[e] = u.z1[e] = u.x0[e] = u.x1[e] = C(0);
  };
  auto aux_load = [&](uint32_t rb, int k, int qy, int qz, int qx, Aux& u) __attribute__((always_inline)) {
    if (iny) ld_pair(rb + yso(k, qy), u.y0, u.y1);
    if (in_z(k)) ld_pair(rb + zso(k, qz), u.z0, u.z1);
    if (lane_inx) ld_xpair(rb + xso(k, qx), u.x0, u.x1);
  };
  auto aux_store = [&](uint32_t rb, int k, int qy, int qz, int qx, const Aux& u) __attribute__((always_inline)) {
    if (iny) st_pair(rb + yso(k, qy), u.y0, u.y1);
    if (in_z(k)) st_pair(rb + zso(k, qz), u.z0, u.z1);
    if (lane_inx) st_xpair(rb + xso(k, qx), u.x0, u.x1);
  };

  // H half step of one row (stages A and C): h <- h - (dt/mu0) curl E with the
  // CPML terms of plane k (z profile index kq); E own samples (ex, ey, ez), the
  // row above (exu, ezu), the plane above (exz, eyz); u: H-side auxiliaries.
  auto h_half = [&](const C (&ex)[V], const C (&ey)[V], const C (&ez)[V], const C (&exu)[V], const C (&ezu)[V],
                    const C (&exz)[V], const C (&eyz)[V], const C (&hx)[V], const C (&hy)[V], const C (&hz)[V],
                    bool inz, int kq, Aux& u, C (&out)[3][V], C eys, C ezs) __attribute__((always_inline)) {
    C eyr[V], ezr[V];
#pragma unroll
    for (int e = 0; e < V - 1; ++e) { eyr[e] = ey[e + 1]; ezr[e] = ez[e + 1]; }
    eyr[V - 1] = from_next_lane(ey[0]);
    ezr[V - 1] = from_next_lane(ez[0]);
    if (seam_hi) { eyr[V - 1] = eys; ezr[V - 1] = ezs; }
    C dEz_dy[V], dEy_dz[V], dEx_dz[V], dEz_dx[V], dEy_dx[V], dEx_dy[V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
      dEz_dy[e] = fdiff(ezu[e], ez[e], idy);
      dEy_dz[e] = fdiff(eyz[e], ey[e], idz);
      dEx_dz[e] = fdiff(exz[e], ex[e], idz);
      dEz_dx[e] = fdiff(ezr[e], ez[e], idx_);
      dEy_dx[e] = fdiff(eyr[e], ey[e], idx_);
      dEx_dy[e] = fdiff(exu[e], ex[e], idy);
    }
    if (iny) {
      const C ob = typ[3 * NW + wv], av = typ[4 * NW + wv], kv = typ[5 * NW + wv];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        dEz_dy[e] = cpml_term(u.y0[e], dEz_dy[e], ob, av, kv);
        dEx_dy[e] = cpml_term(u.y1[e], dEx_dy[e], ob, av, kv);
      }
    }
    if (inz) {
      const C ob = tzp[3 * npl + kq], av = tzp[4 * npl + kq], kv = tzp[5 * npl + kq];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        dEy_dz[e] = cpml_term(u.z0[e], dEy_dz[e], ob, av, kv);
        dEx_dz[e] = cpml_term(u.z1[e], dEx_dz[e], ob, av, kv);
      }
    }
    if (Lx > 0) {
      // lanes outside the layer read (1 - b, a, 1/kappa) = (0, 0, 1) and psi 0
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const int i = xl + e;
        const C ob = txp[3 * RL + i], av = txp[4 * RL + i], kv = txp[5 * RL + i];
        dEz_dx[e] = cpml_term(u.x0[e], dEz_dx[e], ob, av, kv);
        dEy_dx[e] = cpml_term(u.x1[e], dEy_dx[e], ob, av, kv);
      }
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
      out[0][e] = to_storage<T, C>(h_new(hx[e], dEz_dy[e], dEy_dz[e], dtm), a.enc[3], a.dec[3]);
      out[1][e] = to_storage<T, C>(h_new(hy[e], dEx_dz[e], dEz_dx[e], dtm), a.enc[4], a.dec[4]);
      out[2][e] = to_storage<T, C>(h_new(hz[e], dEy_dx[e], dEx_dy[e], dtm), a.enc[5], a.dec[5]);
    }
    if (!lane_ok) {   // lanes beyond nx hold zeros (the x+1 neighbour of the last sample)
#pragma unroll
      for (int e = 0; e < V; ++e) { out[0][e] = C(0); out[1][e] = C(0); out[2][e] = C(0); }
    }
  };

  // E half step of one row at plane k (stages B and D): e <- Ca e + Cb curl H,
  // then the walls, the soft sources of step n+1+s and storage rounding.  H own
  // samples (hx, hy, hz), the row below (hxd, hzd), the plane below (hxz, hyz).
  auto e_half = [&](const C (&ex)[V], const C (&ey)[V], const C (&ez)[V], const C (&hx)[V], const C (&hy)[V],
                    const C (&hz)[V], const C (&hxd)[V], const C (&hzd)[V], const C (&hxz)[V], const C (&hyz)[V],
                    int k, bool inz, int kq, const Coef2<C> (&cf)[V], int pl, uint32_t pm, int s, Aux& u,
                    C (&out)[3][V], C hys, C hzs) __attribute__((always_inline)) {
    C hyl[V], hzl[V];
#pragma unroll
    for (int e = 1; e < V; ++e) { hyl[e] = hy[e - 1]; hzl[e] = hz[e - 1]; }
    hyl[0] = from_prev_lane(hy[V - 1]);
    hzl[0] = from_prev_lane(hz[V - 1]);
    if (seam_lo) { hyl[0] = hys; hzl[0] = hzs; }
    C dHz_dy[V], dHy_dz[V], dHx_dz[V], dHz_dx[V], dHy_dx[V], dHx_dy[V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
      dHz_dy[e] = fdiff(hz[e], hzd[e], idy);
      dHy_dz[e] = fdiff(hy[e], hyz[e], idz);
      dHx_dz[e] = fdiff(hx[e], hxz[e], idz);
      dHz_dx[e] = fdiff(hz[e], hzl[e], idx_);
      dHy_dx[e] = fdiff(hy[e], hyl[e], idx_);
      dHx_dy[e] = fdiff(hx[e], hxd[e], idy);
    }
    if (iny) {
      const C ob = typ[0 * NW + wv], av = typ[1 * NW + wv], kv = typ[2 * NW + wv];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        dHz_dy[e] = cpml_term(u.y0[e], dHz_dy[e], ob, av, kv);
        dHx_dy[e] = cpml_term(u.y1[e], dHx_dy[e], ob, av, kv);
      }
    }
    if (inz) {
      const C ob = tzp[0 * npl + kq], av = tzp[1 * npl + kq], kv = tzp[2 * npl + kq];
#pragma unroll
      for (int e = 0; e < V; ++e) {
        dHy_dz[e] = cpml_term(u.z0[e], dHy_dz[e], ob, av, kv);
        dHx_dz[e] = cpml_term(u.z1[e], dHx_dz[e], ob, av, kv);
      }
    }
    if (Lx > 0) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        const int i = xl + e;
        const C ob = txp[0 * RL + i], av = txp[1 * RL + i], kv = txp[2 * RL + i];
        dHz_dx[e] = cpml_term(u.x0[e], dHz_dx[e], ob, av, kv);
        dHy_dx[e] = cpml_term(u.x1[e], dHy_dx[e], ob, av, kv);
      }
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
      C cax = cf[e].ca, cbx = cf[e].cb, cay = cax, cby = cbx, caz = cax, cbz = cbx;
      if (pl >= 0) {
        const uint32_t m = pm >> (8 * e);
        if (m & 1) { cax = C(0); cbx = C(0); }
        if (m & 2) { cay = C(0); cby = C(0); }
        if (m & 4) { caz = C(0); cbz = C(0); }
      }
      out[0][e] = e_new(ex[e], dHz_dy[e], dHy_dz[e], cax, cbx);
      out[1][e] = e_new(ey[e], dHx_dz[e], dHz_dx[e], cay, cby);
      out[2][e] = e_new(ez[e], dHy_dx[e], dHx_dy[e], caz, cbz);
    }
    // E samples on the outer faces (and beyond nx) are never updated; their
    // auxiliaries stay 0.  Pairs: y (XY, ZY), z (XZ, YZ), x (YX, ZX).
    if (!(j > 0 && k > 0)) {
#pragma unroll
      for (int e = 0; e < V; ++e) { out[0][e] = ex[e]; u.y0[e] = C(0); u.z0[e] = C(0); }
    }
    if (!(k > 0)) {
#pragma unroll
      for (int e = 0; e < V; ++e) { out[1][e] = ey[e]; u.z1[e] = C(0); u.x0[e] = C(0); }
    }
    if (!(j > 0)) {
#pragma unroll
      for (int e = 0; e < V; ++e) { out[2][e] = ez[e]; u.x1[e] = C(0); u.y1[e] = C(0); }
    }
    if (RL > nx) {
#pragma unroll
      for (int e = 0; e < V; ++e)
        if (xl + e >= nx) {
          out[0][e] = ex[e]; out[1][e] = ey[e]; out[2][e] = ez[e];
          u.y0[e] = u.y1[e] = u.z0[e] = u.z1[e] = u.x0[e] = u.x1[e] = C(0);
        }
    }
    if (xl == 0) {   // i = 0: Ey and Ez on the outer face
      out[1][0] = ey[0];
      out[2][0] = ez[0];
      u.z1[0] = C(0); u.x0[0] = C(0); u.x1[0] = C(0); u.y1[0] = C(0);
    }
    const uint8_t fl = tfl[wv * npl + kq];
    if (fl & 1) {
      for (int q = 0; q < a.nsrc; ++q) {
        const SrcDev sp = a.src[q];
        if (sp.j == j && sp.k == k) {
          const C v = ldsS[s * kMaxSources + q];
#pragma unroll
          for (int e = 0; e < V; ++e)
            if (xl + e == sp.i) add_to_comp<C, V>(out, sp.comp, e, v);
        }
      }
    }
#pragma unroll
    for (int e = 0; e < V; ++e) {
      out[0][e] = to_storage<T, C>(out[0][e], a.enc[0], a.dec[0]);
      out[1][e] = to_storage<T, C>(out[1][e], a.enc[1], a.dec[1]);
      out[2][e] = to_storage<T, C>(out[2][e], a.enc[2], a.dec[2]);
    }
  };
  // probe samples of a step on the tile's own samples (row flag bit 1)
  auto record = [&](int k, int kq, const C (&ef)[3][V], const C (&hf)[3][V], int slot) __attribute__((always_inline)) {
    if (tfl[wv * npl + kq] & 2) {
      for (int pp = 0; pp < a.nprobe; ++pp) {
        const int4 pr = a.probe[pp];
        if (pr.z == j && pr.w == k) {
#pragma unroll
          for (int e = 0; e < V; ++e)
            if (xl + e == pr.y) a.series[(size_t)slot * a.nprobe + pp] = static_cast<double>(pick_comp<C, V>(ef, hf, pr.x, e));
        }
      }
    }
  };

  // the row's slots in the parity buffers (computed, not indexed: no private arrays)
  C* const myX0 = X0 + wv * 2 * RL + xl;        // + 0: Ez, + RL: Ex; parity 1 at + NR * 2 * RL
  C* const myHA0 = HA0 + wv * 3 * RL + xl;      // Hx, Hy, Hz; parity 1 at + NW * 3 * RL
  auto myX = [&](int pr) __attribute__((always_inline)) { return myX0 + pr * (NR * 2 * RL); };
  auto myHA = [&](int pr) __attribute__((always_inline)) { return myHA0 + pr * (NW * 3 * RL); };
  C* myHb = Hb + wv * 2 * RL + xl;                                           // + 0: Hz, + RL: Hx
  // seam values of this row: row starts of the LDS rows plus the seam sample
  C* const rowX0 = X0 + wv * 2 * RL;            // Ez of the row at + XS
  C* const rowHA0 = HA0 + wv * 3 * RL;          // Hy at + RL + XS - 1, Hz at + 2 RL + XS - 1
  C* const rowHb = Hb + wv * 2 * RL;            // Hz at + XS - 1
  auto seamEy = [&](int kind, int pr) __attribute__((always_inline)) { return seam + (2 * kind + pr) * NR + wv; };
  C* const seamHy = seam + 4 * NR + wv;

  // (Ca, Cb) of the row's samples at plane k and its PEC mask bytes
  auto load_coef = [&](int kq, Coef2<C> (&cf)[V]) __attribute__((always_inline)) {
    const uint32_t cso = (uint32_t)uniform(tzs[kq]) * (uint32_t)sizeof(Coef2<C>);
#pragma unroll
    for (int e = 0; e < V; ++e) cf[e] = buf_ld<Coef2<C>>(rcoef, vcf[e], cso);
  };
  auto load_mask = [&](int pl) __attribute__((always_inline)) {
    uint32_t pm = 0u;
    if (pl >= 0 && lane_ok) {
      const uint8_t* mb = a.pec_mask + ((size_t)pl * ny + jc) * px + xl;
#pragma unroll
      for (int e = 0; e < V; ++e) pm |= (uint32_t)mb[e] << (8 * e);
    }
    return pm;
  };

  // x-layer auxiliaries between the two steps: through LDS (H side in slots
  // 0, 1; E side in 2, 3), each lane reading back what it wrote
  auto px_put = [&](int pr, int c0, const C (&v0)[V], const C (&v1)[V]) __attribute__((always_inline)) {
    C* b = PX + pr * (NW * 4 * XW) + wv * 4 * XW;
#pragma unroll
    for (int e = 0; e < V; ++e)
      if (xs_slot[e] >= 0) {
        b[c0 * XW + xs_slot[e]] = v0[e];
        b[(c0 + 1) * XW + xs_slot[e]] = v1[e];
      }
  };
  auto px_get = [&](int pr, int c0, C (&v0)[V], C (&v1)[V]) __attribute__((always_inline)) {
    const C* b = PX + pr * (NW * 4 * XW) + wv * 4 * XW;
#pragma unroll
    for (int e = 0; e < V; ++e) {
      v0[e] = xs_slot[e] >= 0 ? b[c0 * XW + xs_slot[e]] : C(0);
      v1[e] = xs_slot[e] >= 0 ? b[(c0 + 1) * XW + xs_slot[e]] : C(0);
    }
  };

  // y- and z-layer auxiliaries between the two steps (slot c0: H side at 0,
  // E side at 4)
  C* const myHO = HO + wv * 8 * RL + xl;
  auto ho_put = [&](int c0, int k, const Aux& u) __attribute__((always_inline)) {
    if (iny) { lds_put<C, V>(myHO + c0 * RL, u.y0); lds_put<C, V>(myHO + (c0 + 1) * RL, u.y1); }
    if (in_z(k)) { lds_put<C, V>(myHO + (c0 + 2) * RL, u.z0); lds_put<C, V>(myHO + (c0 + 3) * RL, u.z1); }
  };
  auto ho_get = [&](int c0, int k, Aux& u) __attribute__((always_inline)) {
    if (iny) { lds_get<C, V>(myHO + c0 * RL, u.y0); lds_get<C, V>(myHO + (c0 + 1) * RL, u.y1); }
    if (in_z(k)) { lds_get<C, V>(myHO + (c0 + 2) * RL, u.z0); lds_get<C, V>(myHO + (c0 + 3) * RL, u.z1); }
  };

  // Memory operations are ordered by need: gfx9 counts outstanding vector
  // loads and stores in one in-order counter, so waiting for a load also waits
  // for everything issued before it.  The old H-side auxiliaries of plane p
  // are loaded before the first barrier, the E-side ones after stage A, then
  // the plane prefetch.  Between the two steps the auxiliaries stay in LDS: the
  // y- and z-layer ones of plane p in the row's slots once the second step of
  // plane p-1 has read its own, the x-layer ones by plane parity.
  auto march = [&](auto role) __attribute__((always_inline)) {
    constexpr int R = decltype(role)::value;
    constexpr bool BOTTOM = R == 0, TOP = R == 2, MID = R == 1;
    const uint32_t vtop = (TOP && jt < ny && lane_ok) ? ((uint32_t)jt * (uint32_t)px + (uint32_t)xl) * TB : kOut;
    C e0y[V], e1[3][V], e2[3][V], h0[3][V], h1[3][V];
    C eByp[V], hCp[2][V];
    C tp1[2][V];   // top role: row j0+ty+1 at plane p+1 (Ex, Ez)
    C e0[3][V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        e0[c][e] = C(0); e1[c][e] = C(0); e2[c][e] = C(0); h0[c][e] = C(0); h1[c][e] = C(0);
      }
      tp1[0][e] = tp1[1][e] = C(0);
      e0y[e] = C(0); eByp[e] = C(0); hCp[0][e] = C(0); hCp[1][e] = C(0);
    }
    load_E(vrow, pbeg, e0);
    load_E(vrow, pbeg + 1, e1);
    load_H(pbeg, h0);
    if constexpr (TOP) load_ExEz(vtop, pbeg, tp1);
    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): the prologue's loads land before the march
    // publish E^n(pbeg) for the first stage A
    lds_put<C, V>(myX(pbeg & 1), e0[2]);
    lds_put<C, V>(myX(pbeg & 1) + RL, e0[0]);
    if constexpr (TOP) {
      lds_put<C, V>(myX(pbeg & 1) + 2 * RL, tp1[1]);
      lds_put<C, V>(myX(pbeg & 1) + 3 * RL, tp1[0]);
    }
#pragma unroll
    for (int e = 0; e < V; ++e) e0y[e] = e0[1][e];
    if (seam_lo) *seamEy(0, pbeg & 1) = e0[1][0];
    // old auxiliaries of the first plane (H side for stage A, E side for B)
    Aux uA, uB;

    for (int p = pbeg; p <= k1; ++p) {
      const int q = p - pbeg;
      const int par = p & 1;
      const bool doA = rowA && p < nz;
      const bool doB = !BOTTOM && doA && p >= k0 - 1;
      const bool doC = MID && rowC && p >= k0 && p >= 1;
      const bool doD = MID && rowD && p >= k0 + 1;
      // old H-side auxiliaries of plane p (their wait also covers the last
      // plane's stores)
      aux_zero(uA);
      if (doA) aux_load(ph_in, p, PHXY, PHXZ, PHYX, uA);
      __syncthreads();   // E^n(p) rows published

      // ---- stage A: H^{n+1/2}(p) of rows j0-2 .. j0+ty ----
      C hA[3][V];
#pragma unroll
      for (int e = 0; e < V; ++e) { hA[0][e] = C(0); hA[1][e] = C(0); hA[2][e] = C(0); }
      if (doA) {
        C ex[V], ez[V], exu[V], ezu[V];
        lds_get<C, V>(myX(par), ez);
        lds_get<C, V>(myX(par) + RL, ex);
        lds_get<C, V>(myX(par) + 2 * RL, ezu);
        lds_get<C, V>(myX(par) + 3 * RL, exu);
        C eys = C(0), ezs = C(0);
        if constexpr (WPR == 2) { eys = *seamEy(0, par); ezs = rowX0[par * (NR * 2 * RL) + XS]; }
        h_half(ex, e0y, ez, exu, ezu, e1[0], e1[1], h0[0], h0[1], h0[2], in_z(p), q, uA, hA, eys, ezs);
        // stage C takes plane p at the next plane
        if constexpr (MID) { if (rowC && p < k1) px_put(par, 0, uA.x0, uA.x1); }
      }
      Coef2<C> cfB[V];
      int plB = -1;
      aux_zero(uB);
      if constexpr (!BOTTOM) {
        if (doB) {
          aux_load(pe_in, p, PEXY, PEXZ, PEYX, uB);
          load_coef(q, cfB);
          plB = uniform(tzl[q]);
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      // ---- the plane prefetch: E^n(p+2), H^{n-1/2}(p+1) (the zero plane past the top) ----
      load_E(vrow, min(p + 2, nz), e2);
      load_H(min(p + 1, nz), h1);
      if constexpr (TOP) load_ExEz(vtop, min(p + 1, nz), tp1);
      __builtin_amdgcn_sched_barrier(0);
      lds_put<C, V>(myHA(par), hA[0]);
      lds_put<C, V>(myHA(par) + RL, hA[1]);
      lds_put<C, V>(myHA(par) + 2 * RL, hA[2]);
      __syncthreads();

      // ---- stage B: E^{n+1}(p) of rows j0-1 .. j0+ty ----
      C eB[3][V];
#pragma unroll
      for (int e = 0; e < V; ++e) { eB[0][e] = C(0); eB[1][e] = C(0); eB[2][e] = C(0); }
      if constexpr (!BOTTOM) {
        if (doB) {
          const uint32_t pmB = load_mask(plB);
          C ex[V], ez[V], hxd[V], hzd[V], hxz[V], hyz[V];
          lds_get<C, V>(myX(par), ez);
          lds_get<C, V>(myX(par) + RL, ex);
          lds_get<C, V>(myHA(par) - 3 * RL, hxd);       // row j-1
          lds_get<C, V>(myHA(par) - RL, hzd);
          lds_get<C, V>(myHA(par ^ 1), hxz);            // plane p-1
          lds_get<C, V>(myHA(par ^ 1) + RL, hyz);
          if (p == 0) {
#pragma unroll
            for (int e = 0; e < V; ++e) { hxz[e] = C(0); hyz[e] = C(0); }
          }
          C hys = C(0), hzs = C(0);
          if constexpr (WPR == 2) {
            hys = rowHA0[par * (NW * 3 * RL) + RL + XS - 1];
            hzs = rowHA0[par * (NW * 3 * RL) + 2 * RL + XS - 1];
          }
          e_half(ex, e0y, ez, hA[0], hA[1], hA[2], hxd, hzd, hxz, hyz, p, in_z(p), q, cfB, plB, pmB, 0, uB, eB, hys,
                 hzs);
          if constexpr (MID) {
            if (rowD && p >= k0 && p < k1) {   // stage D takes plane p at the next plane
              px_put(par, 2, uB.x0, uB.x1);
              record(p, q, eB, hA, a.series_slot);
            }
          }
        }
        lds_put<C, V>(myX(par), eB[2]);
        lds_put<C, V>(myX(par) + RL, eB[0]);
        if (seam_lo) *seamEy(1, par) = eB[1][0];
      }
      __syncthreads();

      // ---- stage C: H^{n+3/2}(p-1) of rows j0-1 .. j0+ty-1 ----
      C hC[3][V];
      Coef2<C> cfD[V];
      int plD = -1;
      if constexpr (MID) {
#pragma unroll
        for (int e = 0; e < V; ++e) { hC[0][e] = C(0); hC[1][e] = C(0); hC[2][e] = C(0); }
        if (doC) {
          Aux uC;
          aux_zero(uC);
          ho_get(0, p - 1, uC);
          px_get(par ^ 1, 0, uC.x0, uC.x1);
          C ex[V], ez[V], exu[V], ezu[V], exz[V], hx[V], hy[V], hz[V];
          lds_get<C, V>(myX(par ^ 1), ez);              // E^{n+1}(p-1)
          lds_get<C, V>(myX(par ^ 1) + RL, ex);
          lds_get<C, V>(myX(par ^ 1) + 2 * RL, ezu);
          lds_get<C, V>(myX(par ^ 1) + 3 * RL, exu);
          lds_get<C, V>(myX(par) + RL, exz);            // E^{n+1}(p): Ex
          lds_get<C, V>(myHA(par ^ 1), hx);             // H^{n+1/2}(p-1)
          lds_get<C, V>(myHA(par ^ 1) + RL, hy);
          lds_get<C, V>(myHA(par ^ 1) + 2 * RL, hz);
          C eys = C(0), ezs = C(0);
          if constexpr (WPR == 2) { eys = *seamEy(1, par ^ 1); ezs = rowX0[(par ^ 1) * (NR * 2 * RL) + XS]; }
          h_half(ex, eByp, ez, exu, ezu, exz, eB[1], hx, hy, hz, in_z(p - 1), q - 1, uC, hC, eys, ezs);
          if (doD) aux_store(ph_out, p - 1, PHXY, PHXZ, PHYX, uC);
        }
        // plane p's first-step H-side auxiliaries replace plane p-1's
        if (rowC && p < k1 && doA) ho_put(0, p, uA);
        lds_put<C, V>(myHb, hC[2]);
        lds_put<C, V>(myHb + RL, hC[0]);
        if (seam_hi) *seamHy = hC[1][V - 1];
        if (doD) {
          load_coef(q - 1, cfD);
          plD = uniform(tzl[q - 1]);
        }
      }
      __syncthreads();

      // ---- stage D: E^{n+2}(p-1) of rows j0 .. j0+ty-1, stores ----
      if constexpr (MID) {
        C eD[3][V];
        C ex[V], ez[V];
        lds_get<C, V>(myX(par ^ 1), ez);
        lds_get<C, V>(myX(par ^ 1) + RL, ex);
#pragma unroll
        for (int e = 0; e < V; ++e) { eD[0][e] = ex[e]; eD[1][e] = eByp[e]; eD[2][e] = ez[e]; }
        Aux uD;
        if (doD) {
          aux_zero(uD);
          ho_get(4, p - 1, uD);
          px_get(par ^ 1, 2, uD.x0, uD.x1);
          const uint32_t pmD = load_mask(plD);
          C hxd[V], hzd[V];
          lds_get<C, V>(myHb - RL, hxd);                // row j-1
          lds_get<C, V>(myHb - 2 * RL, hzd);
          C hys = C(0), hzs = C(0);
          if constexpr (WPR == 2) { hys = *seamHy; hzs = rowHb[XS - 1]; }
          e_half(ex, eByp, ez, hC[0], hC[1], hC[2], hxd, hzd, hCp[0], hCp[1], p - 1, in_z(p - 1), q - 1, cfD, plD,
                 pmD, 1, uD, eD, hys, hzs);
          record(p - 1, q - 1, eD, hC, a.series_slot2);
        }
        // plane p's first-step E-side auxiliaries replace plane p-1's
        if (rowD && p >= k0 && p < k1) ho_put(4, p, uB);
        if (doD) aux_store(pe_out, p - 1, PEXY, PEXZ, PEYX, uD);
        // the field stores are issued at every plane (every lane out of range
        // where nothing is owned), so each iteration issues the same operations
        const uint32_t vst = doD ? vrow : kOut;
        const uint32_t so = (uint32_t)(p >= 1 ? p - 1 : 0) * plane_b;
        st_row<T, C, V>(rout, vst, so, eD[0], a.enc[0], nt);
        st_row<T, C, V>(rout, vst, so + cs_b, eD[1], a.enc[1], nt);
        st_row<T, C, V>(rout, vst, so + 2 * cs_b, eD[2], a.enc[2], nt);
        st_row<T, C, V>(rout, vst, so + 3 * cs_b, hC[0], a.enc[3], nt);
        st_row<T, C, V>(rout, vst, so + 4 * cs_b, hC[1], a.enc[4], nt);
        st_row<T, C, V>(rout, vst, so + 5 * cs_b, hC[2], a.enc[5], nt);
      }

      // ---- publish E^n(p+1) for the next stage A; advance the window ----
      lds_put<C, V>(myX(par ^ 1), e1[2]);
      lds_put<C, V>(myX(par ^ 1) + RL, e1[0]);
      if (seam_lo) *seamEy(0, par ^ 1) = e1[1][0];
      if constexpr (TOP) {
        lds_put<C, V>(myX(par ^ 1) + 2 * RL, tp1[1]);
        lds_put<C, V>(myX(par ^ 1) + 3 * RL, tp1[0]);
      }
#pragma unroll
      for (int e = 0; e < V; ++e) {
        e0y[e] = e1[1][e];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          e1[c][e] = e2[c][e];
          h0[c][e] = h1[c][e];
        }
        if constexpr (MID) {
          eByp[e] = eB[1][e];
          hCp[0][e] = hC[0][e];
          hCp[1][e] = hC[1][e];
        }
      }
    }
  };
  if (wv == 0) march(TbRole<0>{});
  else if (wv == NW - 1) march(TbRole<2>{});
  else march(TbRole<1>{});
}

// Workgroup size the two-step kernel is built for: rows of one wave with two
// samples per lane or fewer, and rows of two waves, take up to 16 waves (four
// per SIMD, at most 128 VGPRs); four samples per lane take 12 (three per SIMD,
// up to 168 VGPRs).
__host__ __device__ constexpr int tb_block_waves(int V) { return V >= 4 ? 12 : 16; }

template <class T, class C, int V, int WPR, bool NT = false>
__global__ void __launch_bounds__(kWave * tb_block_waves(V))
tb_kernel(const StepArgs<T, C> a) {
  extern __shared__ unsigned char smem_raw[];
  // XCD-aware tile order, as in step_kernel: each XCD gets a contiguous run
  // of tiles (neighbouring y-tiles of one z-chunk share halo rows in its L2)
  const int per_xcd = gridDim.x >> 3;
  const int t = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (t >= a.ntiles) return;
  const int k0 = (t / a.ny_tiles) * a.kz;
  tb_tile<T, C, V, WPR, NT>(a, t % a.ny_tiles, k0, min(a.nz, k0 + a.kz), smem_raw);
}

}  // namespace yee
