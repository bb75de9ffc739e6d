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
// Memory pipelining.  gfx9 counts outstanding vector loads and stores in one
// in-order counter, so waiting for any load also waits for every operation
// issued before it, and the compiler's wait for a register counts the
// operations issued after its load on the path with the fewest.  Each
// iteration therefore issues its small loads (CPML auxiliaries, material and
// mask data) first and the plane prefetches (E^n(k+2), H^{n-1/2}(k+1)) after
// them; own rows, the halo row and spare waves march in separate loops, each
// issuing the same prefetch and field stores at every plane, so a wait never
// covers more than the operations it needs.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <stdint.h>

namespace yee {

constexpr int kWave = 64;
constexpr int kMaxBlockWaves = 16;   // 1024 threads

// Waves a workgroup may hold at V samples per lane (bounds the registers the
// compiler may give each lane).
// Waves per workgroup the kernel is built for.  The bound also caps registers:
// at 16 waves a kernel gets 128 VGPRs, and the two-sample kernels spill there
// (FP16 storage: 9 VGPRs, FP64: 348); built for 12 waves they get up to 170.
__host__ __device__ constexpr int max_block_waves(int V) { return V >= 4 ? 8 : (V == 2 ? 12 : 16); }
constexpr int kMaxSources = 8;

// psi auxiliaries (E side in place; H side ping-ponged).  The two of one
// CPML axis are stored interleaved, as pairs: y slab (XY, ZY), z slab
// (XZ, YZ), x slab (YX, ZX); psoff[q] is the element offset of the pair array
// holding q, and psi_member(q) its place in the pair.
enum { PEXY = 0, PEXZ, PEYZ, PEYX, PEZX, PEZY };
enum { PHXY = 0, PHXZ, PHYZ, PHYX, PHZX, PHZY };
__host__ __device__ constexpr int psi_member(int q) { return (q == 5 || q == 2 || q == 4) ? 1 : 0; }

template <class C>
struct alignas(2 * sizeof(C)) Pair {
  C a, b;
};

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
  C* pse;                   // E-side psi (single step: updated in place; two-step sweep: old)
  C* pse_out;               // E-side psi, new (two-step sweep only)
  const C* psbase;          // two-step sweep: lowest of the four auxiliary regions
  uint32_t psi_span;        //                 bytes from psbase to the end of the highest
  const C* psh_in;          // H-side psi, old
  C* psh_out;               // H-side psi, new
  uint32_t psoff[6];        // element offset of the pair array holding each psi auxiliary
  const C* prof;            // CPML profiles [side E,H][axis][1 - b | a | 1/kappa][plen]
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
  int32_t series_slot2;     // ring slot of the second step of a two-step sweep
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
  uint32_t psi_bytes;       // bytes of one psi region (E side; each H-side set is as large)
  uint32_t coef_bytes;      // bytes of the (Ca, Cb) table
  // E^{n+1} of a box of cells (adjoint history; kernels instantiated with it):
  // component c of cell (i, j, k) at hist[c * hstride + ((k - k0) * by + j - j0) * bx + i - i0]
  T* hist;
  uint64_t hstride;
  int32_t hbox[6];          // i0, i1, j0, j1, k0, k1
  // debug (kernels instantiated with it): one count per stored element of the
  // output field set, component c at wcount + c * cstride, incremented by
  // every store of that element (tile ownership: exactly one per step)
  uint32_t* wcount;
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

// ---------------------------------------------------------------------------
// Per-sample arithmetic of one step, shared by every kernel that advances the
// fields (single step, two steps per sweep, batched).  The library is built
// with -ffp-contract=off, so each operation below is exactly the instruction
// written: the same sample gets the same bits whichever kernel computes it.
// ---------------------------------------------------------------------------
// forward or backward difference (hi - lo) / dw
template <class C>
__device__ __forceinline__ C fdiff(C hi, C lo, C inv) { return (hi - lo) * inv; }
// CPML (Roden & Gedney 2000): psi <- b psi + a d, evaluated as
// psi - (1 - b) psi + a d; returns d / kappa + psi
template <class C>
__device__ __forceinline__ C cpml_term(C& psi, C d, C omb, C a, C kinv) {
  psi = fma(a, d, fma(-omb, psi, psi));
  return fma(kinv, d, psi);
}
// H half step: h - (dt/mu0) (p - q)
template <class C>
__device__ __forceinline__ C h_new(C h, C p, C q, C dtm) { return fma(-dtm, p - q, h); }
// E half step (Taflove & Hagness ch. 3): Ca e + Cb (p - q)
template <class C>
__device__ __forceinline__ C e_new(C e, C p, C q, C ca, C cb) { return fma(ca, e, cb * (p - q)); }

template <class T, int V>
struct alignas(sizeof(T) * V) VecT {
  T v[V];
};

// Round a computed value to what storage would hold (identity unless FP16).
template <class T, class C>
__device__ __forceinline__ C to_storage(C v, float enc, float dec) {
  return Conv<T, C>::ld(Conv<T, C>::st(v, enc), dec);
}
// The same, also handing back the storage bits for FP16 storage (stored as
// they are: encoding the decoded value again would give the same bits).  With
// T == C the caller stores the value itself and bits is left alone.
template <class T, class C>
__device__ __forceinline__ C to_storage(C v, float enc, float dec, T& bits) {
  if constexpr (std::is_same<T, C>::value) {
    return v;
  } else {
    bits = Conv<T, C>::st(v, enc);
    return Conv<T, C>::ld(bits, dec);
  }
}

// Source waveform in FP64: w(t) = -2u exp(-u^2) or sin(2 pi f0 (t - t0)) exp(-u^2).
__device__ __noinline__ double waveform(const SrcDev s, double t) {
  const double u = (t - s.t0) / s.tau;
  const double g = exp(-u * u);
  if (s.kind == 0) return -2.0 * u * g;
  return sin(2.0 * M_PI * s.f0 * (t - s.t0)) * g;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Wave role of the march (0 own rows, 1 halo row, 2 spare), as a type.
template <int N>
struct Role {
  static constexpr int value = N;
};

// LDS layout of one workgroup, in compute-type elements unless noted:
//   E rows j0-1 .. j0+ty        [ty+2][3][RS]  (RS = wpr*64*V + 2V: one zero
//   H rows j0-1 .. j0+ty-1      [ty+1][3][RS]   pad vector on each side of a row)
//   source values               [kMaxSources]
//   z profiles of the chunk     [6][kz+1]      (1 - b, a, 1/kappa of the E side, then H side)
//   x profiles                  [6][wpr*64*V]
//   y profiles of the tile rows [6][ty+1]
//   int32: z block offset [kz+1], PEC plane index [kz+1]; uint8: row flags [ty+1][kz+1]
__host__ __device__ inline size_t step_lds_bytes_for(int ty, int wpr, int V, int kz, size_t csize) {
  const size_t rl = (size_t)wpr * kWave * V;
  const size_t rs = rl + 2 * (size_t)V;
  const size_t nk = (size_t)kz + 1;
  size_t b = ((size_t)(2 * ty + 3) * 3 * rs + kMaxSources + 6 * nk + 6 * rl + 6 * (size_t)(ty + 1)) * csize;
  b += 2 * nk * sizeof(int32_t);
  b += (size_t)(ty + 1) * nk;
  return (b + 15) & ~size_t(15);
}

template <class C, int V>
__device__ __forceinline__ void lds_put(C* p, const C (&v)[V]) {
  VecT<C, V> t;
#pragma unroll
  for (int e = 0; e < V; ++e) t.v[e] = v[e];
  *reinterpret_cast<VecT<C, V>*>(p) = t;
}

template <class C, int V>
__device__ __forceinline__ void lds_get(const C* p, C (&v)[V]) {
  const VecT<C, V> t = *reinterpret_cast<const VecT<C, V>*>(p);
#pragma unroll
  for (int e = 0; e < V; ++e) v[e] = t.v[e];
}

// Buffer resources (V#): a base address, a byte range and the gfx9 data
// format word.  Every load and store of the step goes through one of them
// with a per-lane byte offset that stays fixed over the march (VGPR) and a
// uniform byte offset (SGPR), so no lane does 64-bit address arithmetic.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
using rsrc_t = __amdgpu_buffer_rsrc_t;

__device__ __forceinline__ rsrc_t make_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, (int)bytes, 0x00020000);
}

template <int N>
struct Raw;
template <>
struct Raw<2> {
  struct U { unsigned short x; };
  static __device__ __forceinline__ U ld(rsrc_t r, uint32_t vo, uint32_t so) {
    return U{__builtin_amdgcn_raw_buffer_load_b16(r, vo, so, 0)};
  }
  static __device__ __forceinline__ void st(U v, rsrc_t r, uint32_t vo, uint32_t so, bool nt) {
    if (nt)
      __builtin_amdgcn_raw_buffer_store_b16(v.x, r, vo, so, 2);
    else
      __builtin_amdgcn_raw_buffer_store_b16(v.x, r, vo, so, 0);
  }
};
template <>
struct Raw<4> {
  struct U { unsigned int x; };
  static __device__ __forceinline__ U ld(rsrc_t r, uint32_t vo, uint32_t so) {
    return U{__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0)};
  }
  static __device__ __forceinline__ void st(U v, rsrc_t r, uint32_t vo, uint32_t so, bool nt) {
    if (nt)
      __builtin_amdgcn_raw_buffer_store_b32(v.x, r, vo, so, 2);
    else
      __builtin_amdgcn_raw_buffer_store_b32(v.x, r, vo, so, 0);
  }
};
template <>
struct Raw<8> {
  struct U { u32x2 x; };
  static __device__ __forceinline__ U ld(rsrc_t r, uint32_t vo, uint32_t so) {
    return U{__builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0)};
  }
  static __device__ __forceinline__ void st(U v, rsrc_t r, uint32_t vo, uint32_t so, bool nt) {
    if (nt)
      __builtin_amdgcn_raw_buffer_store_b64(v.x, r, vo, so, 2);
    else
      __builtin_amdgcn_raw_buffer_store_b64(v.x, r, vo, so, 0);
  }
};
template <>
struct Raw<16> {
  struct U { u32x4 x; };
  static __device__ __forceinline__ U ld(rsrc_t r, uint32_t vo, uint32_t so) {
    return U{__builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0)};
  }
  static __device__ __forceinline__ void st(U v, rsrc_t r, uint32_t vo, uint32_t so, bool nt) {
    if (nt)
      __builtin_amdgcn_raw_buffer_store_b128(v.x, r, vo, so, 2);
    else
      __builtin_amdgcn_raw_buffer_store_b128(v.x, r, vo, so, 0);
  }
};
template <>
struct Raw<32> {
  struct U { u32x4 x, y; };
  static __device__ __forceinline__ U ld(rsrc_t r, uint32_t vo, uint32_t so) {
    return U{__builtin_amdgcn_raw_buffer_load_b128(r, vo, so, 0), __builtin_amdgcn_raw_buffer_load_b128(r, vo + 16, so, 0)};
  }
  static __device__ __forceinline__ void st(U v, rsrc_t r, uint32_t vo, uint32_t so, bool nt) {
    Raw<16>::st(Raw<16>::U{v.x}, r, vo, so, nt);
    Raw<16>::st(Raw<16>::U{v.y}, r, vo + 16, so, nt);
  }
};

template <class X>
__device__ __forceinline__ X buf_ld(rsrc_t r, uint32_t vo, uint32_t so) {
  using R = Raw<sizeof(X)>;
  return __builtin_bit_cast(X, R::ld(r, vo, so));
}
// Cache policy of a store: nt marks it non-temporal (streamed past the
// last-level cache); a compile-time choice, so each kernel has one store path.
template <class X>
__device__ __forceinline__ void buf_st(const X& v, rsrc_t r, uint32_t vo, uint32_t so, bool nt = false) {
  using R = Raw<sizeof(X)>;
  R::st(__builtin_bit_cast(typename R::U, v), r, vo, so, nt);
}

template <class T, class C, int V>
__device__ __forceinline__ void ld_row(rsrc_t r, uint32_t vo, uint32_t so, C (&out)[V], float dec) {
  const VecT<T, V> v = buf_ld<VecT<T, V>>(r, vo, so);
#pragma unroll
  for (int e = 0; e < V; ++e) out[e] = Conv<T, C>::ld(v.v[e], dec);
}

template <class T, class C, int V>
__device__ __forceinline__ void st_row(rsrc_t r, uint32_t vo, uint32_t so, const C (&in)[V], float enc,
                                       bool nt = false) {
  VecT<T, V> v;
#pragma unroll
  for (int e = 0; e < V; ++e) v.v[e] = Conv<T, C>::st(in[e], enc);
  buf_st<VecT<T, V>>(v, r, vo, so, nt);
}

template <class T, class C, int V>
__device__ __forceinline__ void decode_row(const VecT<T, V>& v, C (&out)[V], float dec) {
#pragma unroll
  for (int e = 0; e < V; ++e) out[e] = Conv<T, C>::ld(v.v[e], dec);
}

// Planes the field prefetch of the fused step runs ahead: two for FP16
// storage with two samples per lane (a wave's loads are then 4 bytes per lane,
// half the bytes in flight of FP32, and the raw values wait packed in one
// register per component), one otherwise (no room in the register budget).
template <class T, int V>
constexpr int prefetch_depth() { return (sizeof(T) == 2 && V == 2) ? 2 : 1; }

// ---------------------------------------------------------------------------
// The fused step: planes [k0, k1) of y-tile ytile of one grid (k1 - k0 <= kz).  Waves beyond
// (ty + 1) * wpr (spare waves of a fixed-size workgroup) take part in the
// barriers only.
//
// Lanes with nothing to load or store (beyond nx, rows outside the grid,
// samples outside an x layer for the x-layer auxiliaries) carry the byte offset
// kOut, outside every buffer range: their loads return 0 and their stores are
// dropped, so the march has no per-lane branches.  Uniform conditions (rows,
// planes, layers) are scalar branches.
//
// Per plane k the registers hold E^n(k), E^n(k+1), H^{n-1/2}(k), H^{n+1/2}(k-1)
// and the H-side psi of plane k.  With a prefetch depth D (prefetch_depth),
// E^n(k+1+D), H^{n-1/2}(k+D) and the row above at k+D are loaded at the top of
// the iteration into a ring of D raw (storage-format) register sets, after the
// small loads the E half waits for (E-side psi and coefficients of plane k):
// gfx9 counts vector memory operations in one in-order counter, so a wait
// never covers a later prefetch.  The set loaded D - 1 iterations earlier is
// decoded into the window at the end of the iteration.  The H-side psi of
// plane k+1 is loaded once plane k's has been consumed.
// ---------------------------------------------------------------------------
constexpr uint32_t kOut = 0x80000000u;

// Extra work of a step_kernel instantiation: none, the adjoint box history,
// or the debug write counts; kStream is the plain step with its field and
// CPML stores streamed past the last-level cache (non-temporal).
enum StepExtra { kPlain = 0, kHistory = 1, kWriteCount = 2, kStream = 3 };

template <class T, class C, int V, int EXTRA = kPlain>
__device__ __forceinline__ void step_tile(const StepArgs<T, C>& a, const int ytile, const int k0,
                                          const int k1, unsigned char* smem_raw) {
  const int wpr = a.wpr;
  const int ty = a.ty;
  constexpr bool nt = EXTRA == kStream;
  const int RL = wpr * kWave * V;
  const int RS = RL + 2 * V;
  const int nk1 = a.kz + 1;
  C* ldsE = reinterpret_cast<C*>(smem_raw);
  C* ldsH = ldsE + (ty + 2) * 3 * RS;
  C* ldsS = ldsH + (ty + 1) * 3 * RS;
  C* tzp = ldsS + kMaxSources;
  C* txp = tzp + 6 * nk1;
  C* typ = txp + 6 * RL;
  int32_t* tzs = reinterpret_cast<int32_t*>(typ + 6 * (ty + 1));
  int32_t* tzl = tzs + nk1;
  uint8_t* tfl = reinterpret_cast<uint8_t*>(tzl + nk1);

  const int nx = a.nx, ny = a.ny, nz = a.nz, px = a.px;
  const int Lx = a.L[0], Ly = a.L[1], Lz = a.L[2];
  const int j0 = ytile * ty;
  const int kstart = k0 > 0 ? k0 - 1 : 0;
  const int nk = k1 - kstart;
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;

  // ---- per-workgroup tables ----
  if (tid < a.nsrc) {
    const SrcDev sd = a.src[tid];
    ldsS[tid] = static_cast<C>(sd.amp * waveform(sd, (double)(a.n + 1) * a.dt));
  }
  for (int q = tid; q < nk; q += nthr) {
    const int k = kstart + q;
    const bool inz = (k < Lz || k >= nz - Lz);
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int side = u / 3, qq = u % 3;
      tzp[u * nk1 + q] = inz ? a.prof[((side * 3 + 2) * 3 + qq) * a.plen + k] : (qq == 2 ? C(1) : C(0));
    }
    tzs[q] = a.seg[px + ny + k] * a.nsxy;
    tzl[q] = a.pec_plane[k];
  }
  for (int q = tid; q < 6 * RL; q += nthr) {
    const int u = q / RL, i = q - u * RL;
    const int side = u / 3, qq = u % 3;
    const bool inx = i < nx && (i < Lx || i >= nx - Lx);
    txp[q] = inx ? a.prof[((side * 3 + 0) * 3 + qq) * a.plen + i] : (qq == 2 ? C(1) : C(0));
  }
  for (int q = tid; q < 6 * (ty + 1); q += nthr) {
    const int u = q / (ty + 1), rr = q - u * (ty + 1);
    const int side = u / 3, qq = u % 3;
    const int jj = j0 - 1 + rr;
    const bool iny = jj >= 0 && jj < ny && (jj < Ly || jj >= ny - Ly);
    typ[q] = iny ? a.prof[((side * 3 + 1) * 3 + qq) * a.plen + jj] : (qq == 2 ? C(1) : C(0));
  }
  for (int q = tid; q < (ty + 1) * nk; q += nthr) {
    const int rr = q / nk, kk = q - rr * nk;
    const int jj = j0 - 1 + rr;
    tfl[rr * nk1 + kk] = (jj >= 0 && jj < ny) ? a.rowflag[(uint32_t)(kstart + kk) * ny + jj] : 0;
  }
  for (int q = tid; q < (2 * ty + 3) * 3 * 2 * V; q += nthr) {
    const int row = q / (2 * V), p = q - row * 2 * V;
    ldsE[row * RS + (p < V ? p : RL + p)] = C(0);
  }
  __syncthreads();

  // ---- wave roles (uniform) ----
  const int wv = uniform(tid >> 6);
  const int lane = tid & 63;
  const bool dummy = wv >= (ty + 1) * wpr;
  const int r = dummy ? 0 : wv / wpr;        // tile row: 0 = halo row j0-1
  const int xs = dummy ? 0 : wv - r * wpr;   // x segment of the row
  const int j = j0 - 1 + r;
  const bool halo = !dummy && r == 0;
  const bool row_ok = !dummy && j >= 0 && j < ny;
  const int jc = min(max(j, 0), ny - 1);
  const bool iny = row_ok && (j < Ly || j >= ny - Ly);
  const int sy = j < Ly ? j : j - ny + 2 * Ly;
  const int jt = j0 + ty;                    // row above the tile
  const bool top_ok = halo && jt < ny;
  const int wx0 = xs * kWave * V;            // first sample of the wave
  const bool wave_inx = row_ok && Lx > 0 && (wx0 < Lx || wx0 + kWave * V > nx - Lx);

  // ---- per-lane offsets (loop invariant; kOut: nothing there) ----
  const int xl = wx0 + lane * V;             // first sample of the lane
  const bool lane_ok = xl < nx;
  constexpr uint32_t TB = sizeof(T), CB = sizeof(C);
  const uint32_t plane = (uint32_t)ny * (uint32_t)px;
  const uint32_t vrow = (row_ok && lane_ok) ? ((uint32_t)jc * (uint32_t)px + (uint32_t)xl) * TB : kOut;
  const uint32_t vtop = (top_ok && lane_ok) ? ((uint32_t)jt * (uint32_t)px + (uint32_t)xl) * TB : kOut;
  const uint32_t vxc = (row_ok && lane_ok) ? (uint32_t)xl * 2 * CB : kOut;   // psi pairs: 2 C per sample
  uint32_t vxs[V], vcf[V];
  const int sx0 = xl < Lx ? xl : xl - nx + 2 * Lx;
  bool lane_inx = false;   // the lane holds x-layer samples: x-slab accesses are exec-masked to
                           // these lanes (out-of-range lanes would still occupy the address unit)
#pragma unroll
  for (int e = 0; e < V; ++e) {
    const int i = xl + e;
    const bool inx = row_ok && i < nx && (i < Lx || i >= nx - Lx);
    lane_inx = lane_inx || inx;
    vxs[e] = inx ? (uint32_t)(sx0 + e) * 2 * CB : kOut;
    vcf[e] = (row_ok && i < nx) ? (uint32_t)(a.seg[i] + a.seg[px + jc] * a.nsx) * (uint32_t)sizeof(Coef2<C>) : kOut;
  }
  const uint32_t plane_b = plane * TB;
  const uint32_t cs_b = (uint32_t)(a.cstride * TB);   // field sets are < 2 GiB (checked on the host)
  const rsrc_t rin = make_rsrc(a.fin, 6 * cs_b);
  const rsrc_t rout = make_rsrc(a.fout, 6 * cs_b);
  const char* psb = reinterpret_cast<const char*>(a.pse);
  const uint32_t phin = (uint32_t)(reinterpret_cast<const char*>(a.psh_in) - psb);
  const uint32_t phout = (uint32_t)(reinterpret_cast<const char*>(a.psh_out) - psb);
  const rsrc_t rpsi = make_rsrc(a.pse, max(phin, phout) + a.psi_bytes);
  const rsrc_t rcoef = make_rsrc(a.coef, a.coef_bytes);
  const C idx_ = a.inv_d[0], idy = a.inv_d[1], idz = a.inv_d[2];
  const C dtm = a.dt_mu;
  // byte offsets (inside a psi region) of plane k of array q in the y, z, x slabs
  auto yso = [&](int k, int q) { return (a.psoff[q] + ((uint32_t)k * (2 * Ly) + sy) * (uint32_t)px * 2) * CB; };
  auto zso = [&](int k, int q) {
    const int sz = k < Lz ? k : k - nz + 2 * Lz;
    return (a.psoff[q] + ((uint32_t)sz * ny + jc) * (uint32_t)px * 2) * CB;
  };
  auto xso = [&](int k, int q) { return (a.psoff[q] + ((uint32_t)k * ny + jc) * (uint32_t)(2 * Lx) * 2) * CB; };
  auto in_z = [&](int k) { return k < Lz || k >= nz - Lz; };

  C* myE = ldsE + r * 3 * RS + V + xl;       // lane's samples in its LDS rows (+ c * RS)
  C* myH = ldsH + r * 3 * RS + V + xl;

  auto load_E = [&](int k, C (&out)[3][V]) {
    const uint32_t so = (uint32_t)k * plane_b;   // k <= nz: plane nz is the zero plane
    ld_row<T, C, V>(rin, vrow, so, out[0], a.dec[0]);
    ld_row<T, C, V>(rin, vrow, so + cs_b, out[1], a.dec[1]);
    ld_row<T, C, V>(rin, vrow, so + 2 * cs_b, out[2], a.dec[2]);
  };
  auto load_E_raw = [&](int k, VecT<T, V> (&out)[3]) {
    const uint32_t so = (uint32_t)k * plane_b;
    out[0] = buf_ld<VecT<T, V>>(rin, vrow, so);
    out[1] = buf_ld<VecT<T, V>>(rin, vrow, so + cs_b);
    out[2] = buf_ld<VecT<T, V>>(rin, vrow, so + 2 * cs_b);
  };
  // Hy of the halo row is not needed; its load is still issued (with every
  // lane out of range), so that every wave issues the same prefetch
  const uint32_t vrow_hy = halo ? kOut : vrow;
  auto load_H = [&](int k, C (&out)[3][V]) {
    const uint32_t so = 3 * cs_b + (uint32_t)k * plane_b;
    ld_row<T, C, V>(rin, vrow, so, out[0], a.dec[3]);
    ld_row<T, C, V>(rin, vrow_hy, so + cs_b, out[1], a.dec[4]);
    ld_row<T, C, V>(rin, vrow, so + 2 * cs_b, out[2], a.dec[5]);
  };
  auto load_H_raw = [&](int k, VecT<T, V> (&out)[3]) {
    const uint32_t so = 3 * cs_b + (uint32_t)k * plane_b;
    out[0] = buf_ld<VecT<T, V>>(rin, vrow, so);
    out[1] = buf_ld<VecT<T, V>>(rin, vrow_hy, so + cs_b);
    out[2] = buf_ld<VecT<T, V>>(rin, vrow, so + 2 * cs_b);
  };
  auto load_top = [&](int k, C (&tz)[V], C (&tx)[V]) {
    if (top_ok) {
      const uint32_t so = (uint32_t)k * plane_b;
      ld_row<T, C, V>(rin, vtop, so + 2 * cs_b, tz, a.dec[2]);
      ld_row<T, C, V>(rin, vtop, so, tx, a.dec[0]);
    }
  };
  auto load_top_raw = [&](int k, VecT<T, V> (&out)[2]) {
    if (top_ok) {
      const uint32_t so = (uint32_t)k * plane_b;
      out[0] = buf_ld<VecT<T, V>>(rin, vtop, so + 2 * cs_b);
      out[1] = buf_ld<VecT<T, V>>(rin, vtop, so);
    }
  };
  C ph[6][V];   // H-side psi of the current plane
  auto load_ph = [&](int k) {
    if (iny) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        { const Pair<C> v_ = buf_ld<Pair<C>>(rpsi, vxc + e * 2 * CB, phin + yso(k, PHXY)); ph[PHXY][e] = v_.a; ph[PHZY][e] = v_.b; }
      }
    }
    if (row_ok && in_z(k)) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        { const Pair<C> v_ = buf_ld<Pair<C>>(rpsi, vxc + e * 2 * CB, phin + zso(k, PHXZ)); ph[PHXZ][e] = v_.a; ph[PHYZ][e] = v_.b; }
      }
    }
    if (wave_inx && lane_inx) {
#pragma unroll
      for (int e = 0; e < V; ++e) {
        { const Pair<C> v_ = buf_ld<Pair<C>>(rpsi, vxs[e], phin + xso(k, PHYX)); ph[PHYX][e] = v_.a; ph[PHZX][e] = v_.b; }
      }
    }
  };

  // ---- prologue: plane kstart ----
  constexpr int D = prefetch_depth<T, V>();
  C e0[3][V], e1[3][V], h0[3][V];
  C hxp[V], hyp[V], tz0[V], tx0[V];
  VecT<T, V> qe[D][3], qh[D][3], qt[D][2];   // prefetch ring (storage format)
  C pe[6][V];
  Coef2<C> cf[V];
  int cf_blk = -1;   // z block offset the coefficients in cf belong to
  uint32_t pm[V];
#pragma unroll
  for (int e = 0; e < V; ++e) {
#pragma unroll
    for (int c = 0; c < 3; ++c) { e0[c][e] = C(0); e1[c][e] = C(0); h0[c][e] = C(0); }
#pragma unroll
    for (int u = 0; u < 6; ++u) { ph[u][e] = C(0); pe[u][e] = C(0); }
    hxp[e] = C(0); hyp[e] = C(0); tz0[e] = C(0); tx0[e] = C(0);
    pm[e] = 0u;
    cf[e].ca = C(0); cf[e].cb = C(0);
#pragma unroll
    for (int d = 0; d < D; ++d) {
#pragma unroll
      for (int c = 0; c < 3; ++c) { qe[d][c].v[e] = T(0); qh[d][c].v[e] = T(0); }
      qt[d][0].v[e] = T(0);
      qt[d][1].v[e] = T(0);
    }
  }
  // Wave roles.  own: a row j0 .. j0+ty-1 inside the grid; halo: row j0-1
  // (its H is recomputed; it also loads the row above the tile); spare: a row
  // beyond the grid (its LDS rows hold zeros, the neighbours of the last row)
  // or a wave beyond the tile.  Each role marches in a loop of its own, whose
  // memory operations are the same at every plane, so that the compiler's
  // count-based waits for a load never cover loads or stores issued after it.
  const bool spare = dummy || (!halo && !row_ok);
  if (!spare) {
    load_ph(kstart);
    load_E(kstart, e0);
    load_E(kstart + 1, e1);
    load_H(kstart, h0);
    load_top(kstart, tz0, tx0);
    if constexpr (D > 1) {
      // the set the first iteration decodes: E^n(kstart+2), H and the row above at kstart+1
      const bool ahead = kstart + 1 < k1;
      load_E_raw(ahead ? kstart + 2 : nz, qe[D - 1]);
      load_H_raw(ahead ? kstart + 1 : nz, qh[D - 1]);
      if (halo) load_top_raw(ahead ? kstart + 1 : nz, qt[D - 1]);
    }
  } else if (!dummy) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lds_put<C, V>(myE + c * RS, e0[c]);
      lds_put<C, V>(myH + c * RS, h0[c]);
    }
  }
  // the prologue's loads land before the march (the wait analysis would
  // otherwise carry them into the loop as pending on the window registers)
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)

  auto march = [&](auto role) {
    constexpr int R = decltype(role)::value;
    constexpr bool OWN = R == 0, HALO = R == 1;
    // one plane; the prefetch goes into ring set S, the window advances from
    // set (S + 1) % D (loaded D - 1 iterations earlier)
    auto iter = [&](const int k, auto slot) __attribute__((always_inline)) {
      constexpr int S = decltype(slot)::value;
      constexpr int SN = (S + 1) % D;
      if constexpr (R == 2) {
        __syncthreads();
        __syncthreads();
        return;
      } else {
      const int kq = k - kstart;
      const bool upd = OWN && k >= k0;      // uniform: this wave updates E and stores at plane k
      const bool more = k + 1 < k1;
      const bool inz = row_ok && in_z(k);
      const int pln = uniform(tzl[kq]);

      // ---- 1. small loads of plane k for the E half ----
      if (upd) {
        if (iny) {
#pragma unroll
          for (int e = 0; e < V; ++e) {
            { const Pair<C> v_ = buf_ld<Pair<C>>(rpsi, vxc + e * 2 * CB, yso(k, PEXY)); pe[PEXY][e] = v_.a; pe[PEZY][e] = v_.b; }
          }
        }
        if (inz) {
#pragma unroll
          for (int e = 0; e < V; ++e) {
            { const Pair<C> v_ = buf_ld<Pair<C>>(rpsi, vxc + e * 2 * CB, zso(k, PEXZ)); pe[PEXZ][e] = v_.a; pe[PEYZ][e] = v_.b; }
          }
        }
        if (wave_inx && lane_inx) {
#pragma unroll
          for (int e = 0; e < V; ++e) {
            { const Pair<C> v_ = buf_ld<Pair<C>>(rpsi, vxs[e], xso(k, PEYX)); pe[PEYX][e] = v_.a; pe[PEZX][e] = v_.b; }
          }
        }
        const int zblk = uniform(tzs[kq]);
        if (zblk != cf_blk) {   // (Ca, Cb) change along z only where the z block does
          cf_blk = zblk;
          const uint32_t cso = (uint32_t)zblk * (uint32_t)sizeof(Coef2<C>);
#pragma unroll
          for (int e = 0; e < V; ++e) cf[e] = buf_ld<Coef2<C>>(rcoef, vcf[e], cso);
        }
        if (pln >= 0) {
          if (lane_ok) {
            const uint8_t* mb = a.pec_mask + ((size_t)pln * ny + jc) * px + xl;
#pragma unroll
            for (int e = 0; e < V; ++e) pm[e] = mb[e];
          }
        }
      }
      __builtin_amdgcn_sched_barrier(0);
      // ---- 2. prefetch E^n(k+1+D), H^{n-1/2}(k+D) and the row above at k+D ----
      // (planes no iteration of the chunk will use: the zero plane)
      {
        const bool ahead = k + D < k1;
        load_E_raw(ahead ? k + 1 + D : nz, qe[S]);
        load_H_raw(ahead ? k + D : nz, qh[S]);
        if constexpr (HALO) load_top_raw(ahead ? k + D : nz, qt[S]);
      }
      __builtin_amdgcn_sched_barrier(0);

      // ---- 3. publish E^n(k) ----
      lds_put<C, V>(myE, e0[0]);
      lds_put<C, V>(myE + RS, e0[1]);
      lds_put<C, V>(myE + 2 * RS, e0[2]);
      if constexpr (HALO) {
        C* rt = ldsE + (ty + 1) * 3 * RS + V + xl;
        lds_put<C, V>(rt, tx0);
        lds_put<C, V>(rt + 2 * RS, tz0);
      }
      __syncthreads();

      // ---- 4. H half step at plane k ----
      C hx[V], hy[V], hz[V];
      VecT<T, V> sh[3];   // H^{n+1/2}(k) in storage format
#pragma unroll
      for (int e = 0; e < V; ++e) {
        hx[e] = C(0); hy[e] = C(0); hz[e] = C(0);
        sh[0].v[e] = T(0); sh[1].v[e] = T(0); sh[2].v[e] = T(0);
      }
      if (OWN || row_ok) {
        C exu[V], ezu[V], eyr[V], ezr[V];
        lds_get<C, V>(myE + 3 * RS, exu);           // row j+1
        lds_get<C, V>(myE + 5 * RS, ezu);
#pragma unroll
        for (int e = 0; e < V - 1; ++e) { eyr[e] = e0[1][e + 1]; ezr[e] = e0[2][e + 1]; }
        eyr[V - 1] = myE[RS + V];                   // x+1 of the last sample (right pad: 0)
        ezr[V - 1] = myE[2 * RS + V];
        C dEz_dy[V], dEy_dz[V], dEx_dz[V], dEz_dx[V], dEy_dx[V], dEx_dy[V];
#pragma unroll
        for (int e = 0; e < V; ++e) {
          dEz_dy[e] = fdiff(ezu[e], e0[2][e], idy);
          dEy_dz[e] = fdiff(e1[1][e], e0[1][e], idz);
          dEx_dz[e] = fdiff(e1[0][e], e0[0][e], idz);
          dEz_dx[e] = fdiff(ezr[e], e0[2][e], idx_);
          dEy_dx[e] = fdiff(eyr[e], e0[1][e], idx_);
          dEx_dy[e] = fdiff(exu[e], e0[0][e], idy);
        }
        if (iny) {
          const C ob = typ[3 * (ty + 1) + r], av = typ[4 * (ty + 1) + r], kv = typ[5 * (ty + 1) + r];
#pragma unroll
          for (int e = 0; e < V; ++e) {
            dEz_dy[e] = cpml_term(ph[PHXY][e], dEz_dy[e], ob, av, kv);
            dEx_dy[e] = cpml_term(ph[PHZY][e], dEx_dy[e], ob, av, kv);
          }
        }
        if (inz) {
          const C ob = tzp[3 * nk1 + kq], av = tzp[4 * nk1 + kq], kv = tzp[5 * nk1 + kq];
#pragma unroll
          for (int e = 0; e < V; ++e) {
            dEy_dz[e] = cpml_term(ph[PHXZ][e], dEy_dz[e], ob, av, kv);
            dEx_dz[e] = cpml_term(ph[PHYZ][e], dEx_dz[e], ob, av, kv);
          }
        }
        if (wave_inx) {
#pragma unroll
          for (int e = 0; e < V; ++e) {
            // lanes outside the layer read (1 - b, a, 1/kappa) = (0, 0, 1) and psi 0
            const int i = xl + e;
            const C ob = txp[3 * RL + i], av = txp[4 * RL + i], kv = txp[5 * RL + i];
            dEz_dx[e] = cpml_term(ph[PHYX][e], dEz_dx[e], ob, av, kv);
            dEy_dx[e] = cpml_term(ph[PHZX][e], dEy_dx[e], ob, av, kv);
          }
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
          hx[e] = to_storage<T, C>(h_new(h0[0][e], dEz_dy[e], dEy_dz[e], dtm), a.enc[3], a.dec[3], sh[0].v[e]);
          hy[e] = HALO ? C(0)
                       : to_storage<T, C>(h_new(h0[1][e], dEx_dz[e], dEz_dx[e], dtm), a.enc[4], a.dec[4], sh[1].v[e]);
          hz[e] = to_storage<T, C>(h_new(h0[2][e], dEy_dx[e], dEx_dy[e], dtm), a.enc[5], a.dec[5], sh[2].v[e]);
        }
        // new H-side psi of the own rows
        if (upd) {
          if (iny) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
              buf_st<Pair<C>>(Pair<C>{ph[PHXY][e], ph[PHZY][e]}, rpsi, vxc + e * 2 * CB, phout + yso(k, PHXY), nt);
            }
          }
          if (inz) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
              buf_st<Pair<C>>(Pair<C>{ph[PHXZ][e], ph[PHYZ][e]}, rpsi, vxc + e * 2 * CB, phout + zso(k, PHXZ), nt);
            }
          }
          if (wave_inx && lane_inx) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
              buf_st<Pair<C>>(Pair<C>{ph[PHYX][e], ph[PHZX][e]}, rpsi, vxs[e], phout + xso(k, PHYX), nt);
            }
          }
        }
      }
      // lanes beyond nx publish zeros (the x+1 neighbour of the last sample)
      if (!lane_ok) {
#pragma unroll
        for (int e = 0; e < V; ++e) { hx[e] = C(0); hy[e] = C(0); hz[e] = C(0); }
      }

      // ---- 5. H-side psi of plane k+1 (its registers are free now; issued
      // before the barrier, which adds the barrier wait to their lead) ----
      if (more) load_ph(k + 1);
      __builtin_amdgcn_sched_barrier(0);

      // ---- 6. publish H^{n+1/2}(k) ----
      lds_put<C, V>(myH, hx);
      lds_put<C, V>(myH + RS, hy);
      lds_put<C, V>(myH + 2 * RS, hz);
      __syncthreads();

      // ---- 7. E half step at plane k and stores ----
      if constexpr (OWN) {
        C exo[V], eyo[V], ezo[V];
        VecT<T, V> se[3];   // E^{n+1}(k) in storage format
#pragma unroll
        for (int e = 0; e < V; ++e) {
          exo[e] = e0[0][e]; eyo[e] = e0[1][e]; ezo[e] = e0[2][e];
          se[0].v[e] = T(0); se[1].v[e] = T(0); se[2].v[e] = T(0);
        }
        uint8_t flags = 0;
        if (upd) {
          C hxd[V], hzd[V], hyl[V], hzl[V];
          lds_get<C, V>(myH - 3 * RS, hxd);             // row j-1
          lds_get<C, V>(myH - RS, hzd);
#pragma unroll
          for (int e = 1; e < V; ++e) { hyl[e] = hy[e - 1]; hzl[e] = hz[e - 1]; }
          hyl[0] = myH[RS - 1];                         // x-1 of the first sample (left pad at i = 0)
          hzl[0] = myH[2 * RS - 1];
          C dHz_dy[V], dHy_dz[V], dHx_dz[V], dHz_dx[V], dHy_dx[V], dHx_dy[V];
#pragma unroll
          for (int e = 0; e < V; ++e) {
            dHz_dy[e] = fdiff(hz[e], hzd[e], idy);
            dHy_dz[e] = fdiff(hy[e], hyp[e], idz);
            dHx_dz[e] = fdiff(hx[e], hxp[e], idz);
            dHz_dx[e] = fdiff(hz[e], hzl[e], idx_);
            dHy_dx[e] = fdiff(hy[e], hyl[e], idx_);
            dHx_dy[e] = fdiff(hx[e], hxd[e], idy);
          }
          if (iny) {
            const C ob = typ[0 * (ty + 1) + r], av = typ[1 * (ty + 1) + r], kv = typ[2 * (ty + 1) + r];
#pragma unroll
            for (int e = 0; e < V; ++e) {
              dHz_dy[e] = cpml_term(pe[PEXY][e], dHz_dy[e], ob, av, kv);
              dHx_dy[e] = cpml_term(pe[PEZY][e], dHx_dy[e], ob, av, kv);
            }
          }
          if (inz) {
            const C ob = tzp[0 * nk1 + kq], av = tzp[1 * nk1 + kq], kv = tzp[2 * nk1 + kq];
#pragma unroll
            for (int e = 0; e < V; ++e) {
              dHy_dz[e] = cpml_term(pe[PEXZ][e], dHy_dz[e], ob, av, kv);
              dHx_dz[e] = cpml_term(pe[PEYZ][e], dHx_dz[e], ob, av, kv);
            }
          }
          if (wave_inx) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
              const int i = xl + e;
              const C ob = txp[0 * RL + i], av = txp[1 * RL + i], kv = txp[2 * RL + i];
              dHz_dx[e] = cpml_term(pe[PEYX][e], dHz_dx[e], ob, av, kv);
              dHy_dx[e] = cpml_term(pe[PEZX][e], dHy_dx[e], ob, av, kv);
            }
          }
          const bool ux = j > 0 && k > 0;     // uniform: Ex off the outer faces
          const bool uy = k > 0;              // uniform part (Ey, Ez also need i > 0)
          const bool uz = j > 0;
#pragma unroll
          for (int e = 0; e < V; ++e) {
            C cax = cf[e].ca, cbx = cf[e].cb, cay = cax, cby = cbx, caz = cax, cbz = cbx;
            if (pln >= 0) {
              const uint32_t m = pm[e];
              if (m & 1) { cax = C(0); cbx = C(0); }
              if (m & 2) { cay = C(0); cby = C(0); }
              if (m & 4) { caz = C(0); cbz = C(0); }
            }
            exo[e] = e_new(e0[0][e], dHz_dy[e], dHy_dz[e], cax, cbx);
            eyo[e] = e_new(e0[1][e], dHx_dz[e], dHz_dx[e], cay, cby);
            ezo[e] = e_new(e0[2][e], dHy_dx[e], dHx_dy[e], caz, cbz);
          }
          if (!ux) {
#pragma unroll
            for (int e = 0; e < V; ++e) { exo[e] = e0[0][e]; pe[PEXY][e] = C(0); pe[PEXZ][e] = C(0); }
          }
          if (!uy) {
#pragma unroll
            for (int e = 0; e < V; ++e) { eyo[e] = e0[1][e]; pe[PEYZ][e] = C(0); pe[PEYX][e] = C(0); }
          }
          if (!uz) {
#pragma unroll
            for (int e = 0; e < V; ++e) { ezo[e] = e0[2][e]; pe[PEZX][e] = C(0); pe[PEZY][e] = C(0); }
          }
          // samples beyond nx in a lane's vector (rows not a multiple of V): never updated
          if (V > 1 && (nx % V) != 0 && wx0 + kWave * V > nx) {
#pragma unroll
            for (int e = 0; e < V; ++e)
              if (xl + e >= nx) {
                exo[e] = e0[0][e]; eyo[e] = e0[1][e]; ezo[e] = e0[2][e];
#pragma unroll
                for (int u = 0; u < 6; ++u) pe[u][e] = C(0);
              }
          }
          // E samples at i = 0 are on the outer face: never updated
          if (xs == 0) {
            if (lane == 0) {
              eyo[0] = e0[1][0];
              ezo[0] = e0[2][0];
              pe[PEYZ][0] = C(0); pe[PEYX][0] = C(0); pe[PEZX][0] = C(0); pe[PEZY][0] = C(0);
            }
          }
          if (iny) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
              buf_st<Pair<C>>(Pair<C>{pe[PEXY][e], pe[PEZY][e]}, rpsi, vxc + e * 2 * CB, yso(k, PEXY), nt);
            }
          }
          if (inz) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
              buf_st<Pair<C>>(Pair<C>{pe[PEXZ][e], pe[PEYZ][e]}, rpsi, vxc + e * 2 * CB, zso(k, PEXZ), nt);
            }
          }
          if (wave_inx && lane_inx) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
              buf_st<Pair<C>>(Pair<C>{pe[PEYX][e], pe[PEZX][e]}, rpsi, vxs[e], xso(k, PEYX), nt);
            }
          }
          flags = tfl[r * nk1 + kq];
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
            exo[e] = to_storage<T, C>(exo[e], a.enc[0], a.dec[0], se[0].v[e]);
            eyo[e] = to_storage<T, C>(eyo[e], a.enc[1], a.dec[1], se[1].v[e]);
            ezo[e] = to_storage<T, C>(ezo[e], a.enc[2], a.dec[2], se[2].v[e]);
          }
        }
        // The field stores are issued at every plane; below the chunk (the
        // warm-up plane, which updates nothing) every lane is out of range.
        const uint32_t vst = upd ? vrow : kOut;
        const uint32_t so = (uint32_t)k * plane_b;
        if constexpr (std::is_same<T, C>::value) {
          st_row<T, C, V>(rout, vst, so, exo, a.enc[0], nt);
          st_row<T, C, V>(rout, vst, so + cs_b, eyo, a.enc[1], nt);
          st_row<T, C, V>(rout, vst, so + 2 * cs_b, ezo, a.enc[2], nt);
          st_row<T, C, V>(rout, vst, so + 3 * cs_b, hx, a.enc[3], nt);
          st_row<T, C, V>(rout, vst, so + 4 * cs_b, hy, a.enc[4], nt);
          st_row<T, C, V>(rout, vst, so + 5 * cs_b, hz, a.enc[5], nt);
        } else {
          buf_st<VecT<T, V>>(se[0], rout, vst, so, nt);
          buf_st<VecT<T, V>>(se[1], rout, vst, so + cs_b, nt);
          buf_st<VecT<T, V>>(se[2], rout, vst, so + 2 * cs_b, nt);
          buf_st<VecT<T, V>>(sh[0], rout, vst, so + 3 * cs_b, nt);
          buf_st<VecT<T, V>>(sh[1], rout, vst, so + 4 * cs_b, nt);
          buf_st<VecT<T, V>>(sh[2], rout, vst, so + 5 * cs_b, nt);
        }
        if constexpr (EXTRA == kWriteCount) {
          if (vst != kOut) {
            const uint32_t o = vst / (uint32_t)sizeof(T) + (uint32_t)k * plane;
#pragma unroll
            for (int e = 0; e < V; ++e)
#pragma unroll
              for (int c = 0; c < 6; ++c) atomicAdd(a.wcount + (size_t)c * a.cstride + o + e, 1u);
          }
        }
        if constexpr (EXTRA == kHistory) {
          // E^{n+1} of the box cells of this row and plane (adjoint history)
          if (upd && j >= a.hbox[2] && j < a.hbox[3] && k >= a.hbox[4] && k < a.hbox[5]) {
            const int hbx = a.hbox[1] - a.hbox[0], hby = a.hbox[3] - a.hbox[2];
            T* hp = a.hist + ((size_t)(k - a.hbox[4]) * hby + (j - a.hbox[2])) * hbx;
#pragma unroll
            for (int e = 0; e < V; ++e) {
              const int i = xl + e;
              if (i >= a.hbox[0] && i < a.hbox[1]) {
                const size_t h = (size_t)(i - a.hbox[0]);
                if constexpr (std::is_same<T, C>::value) {
                  hp[h] = exo[e];
                  hp[a.hstride + h] = eyo[e];
                  hp[2 * a.hstride + h] = ezo[e];
                } else {
                  hp[h] = se[0].v[e];
                  hp[a.hstride + h] = se[1].v[e];
                  hp[2 * a.hstride + h] = se[2].v[e];
                }
              }
            }
          }
        }
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

      // ---- 8. advance the register window ----
      {
        C e2[3][V], h1[3][V];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          decode_row<T, C, V>(qe[SN][c], e2[c], a.dec[c]);
          decode_row<T, C, V>(qh[SN][c], h1[c], a.dec[3 + c]);
        }
        if constexpr (HALO) {
          decode_row<T, C, V>(qt[SN][0], tz0, a.dec[2]);
          decode_row<T, C, V>(qt[SN][1], tx0, a.dec[0]);
        }
#pragma unroll
        for (int e = 0; e < V; ++e) {
          hxp[e] = hx[e];
          hyp[e] = hy[e];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            e0[c][e] = e1[c][e];
            e1[c][e] = e2[c][e];
            h0[c][e] = h1[c][e];
          }
        }
      }
      }
    };
    for (int k = kstart; k < k1; k += D) {
      iter(k, Role<0>{});
      if constexpr (D > 1) {
        if (k + 1 < k1) iter(k + 1, Role<1>{});
      }
    }
  };
  if (spare) march(Role<2>{});
  else if (halo) march(Role<1>{});
  else march(Role<0>{});
}

// ---------------------------------------------------------------------------
// The fused step kernel: one grid, one tile (y-tile, chunk of kz planes) per
// workgroup.  The host picks kz so that every tile fits the device at once
// (one round: no workgroup waits for a slot).
// ---------------------------------------------------------------------------
// Waves per SIMD the step kernel is compiled for.  FP32 arithmetic with one
// sample per lane: six, so that two 12-wave workgroups share a CU (at most 80
// VGPRs); otherwise no bound.
template <class C, int V>
constexpr int step_waves_per_eu() { return (sizeof(C) == 4 && V == 1) ? 6 : 1; }

template <class T, class C, int V, int EXTRA = kPlain>
__global__ void __launch_bounds__(kWave * max_block_waves(V))
__attribute__((amdgpu_waves_per_eu(step_waves_per_eu<C, V>())))
step_kernel(const StepArgs<T, C> a) {
  extern __shared__ unsigned char smem_raw[];
  // XCD-aware tile order: consecutive workgroup ids are dealt round-robin to
  // the 8 XCDs, so give each XCD a contiguous run of tiles (neighbouring
  // y-tiles of one z-chunk, which share halo rows in that XCD's L2).
  const int per_xcd = gridDim.x >> 3;
  const int t = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
  if (t >= a.ntiles) return;
  const int k0 = (t / a.ny_tiles) * a.kz;
  step_tile<T, C, V, EXTRA>(a, t % a.ny_tiles, k0, min(a.nz, k0 + a.kz), smem_raw);
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

template <class T, class C, int V, int EXTRA = kPlain>
__global__ void __launch_bounds__(kWave * max_block_waves(V))
__attribute__((amdgpu_waves_per_eu(step_waves_per_eu<C, V>())))
batch_step_kernel(const SlotDesc<T, C>* __restrict__ slots, const int32_t* __restrict__ hdr, const int q) {
  extern __shared__ unsigned char smem_raw[];
  const int nslots = hdr[0], total = hdr[1];
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int s = 0;
    while (s + 1 < nslots && slots[s + 1].tile0 <= t) ++s;
    const int64_t n = slots[s].base_n + q;
    if (n < slots[s].n_end) {
      StepArgs<T, C> a = slots[s].a;
      const int par = (int)((n - slots[s].base_n) & 1);   // set[0]: the state at the replay's start
      a.fin = slots[s].set[par];
      a.fout = const_cast<T*>(slots[s].set[par ^ 1]);
      a.psh_in = slots[s].psh[par];
      a.psh_out = slots[s].psh[par ^ 1];
      a.n = n;
      a.series_slot = (int32_t)(n % slots[s].series_len);
      const int tl = t - slots[s].tile0;
      const int kb = (tl / a.ny_tiles) * a.kz;
      step_tile<T, C, V, EXTRA>(a, tl % a.ny_tiles, kb, min(a.nz, kb + a.kz), smem_raw);
    }
    __syncthreads();  // the next tile reuses the LDS
  }
}

// ---------------------------------------------------------------------------
// Running DFT fold: one wave per (probe, frequency); lanes stride over the
// samples of the chunk, partial sums meet in a butterfly of lane shuffles.
// X_p(f) += sum_n y_p[n] exp(-i 2 pi f n dt) dt for n = n_first .. n_first+count-1.
// ---------------------------------------------------------------------------
constexpr uint32_t kFlagNonFinite = 1u;   // a NaN or infinity was found
constexpr uint32_t kFlagOverflow = 2u;    // FP16 storage overflowed (an infinity)

// The wave of frequency 0 also checks the probe's samples and sets bit 0 of
// *flags when one is not finite.
__global__ void __launch_bounds__(256)
dft_fold_kernel(const double* __restrict__ series, int nprobe, int series_len, int64_t n_first,
                int count, const double* __restrict__ freqs, int nf, double dt,
                double2* __restrict__ acc, uint32_t* __restrict__ flags) {
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (wid >= nprobe * nf) return;
  const int p = wid / nf;
  const int m = wid % nf;
  const double fdt = freqs[m] * dt;
  double re = 0.0, im = 0.0;
  bool bad = false;
  for (int s = lane; s < count; s += kWave) {
    const int64_t n = n_first + s;                  // 1-based step number
    const double y = series[(size_t)((n - 1) % series_len) * nprobe + p];
    bad |= !isfinite(y);
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
  if (m == 0 && __ballot(bad) != 0 && lane == 0) atomicOr(flags, kFlagNonFinite);
  if (lane == 0) {
    double2 v = acc[wid];
    v.x += re * dt;
    v.y += im * dt;
    acc[wid] = v;
  }
}

// ---------------------------------------------------------------------------
// Status scan: ORs into *flags what it finds in two ranges of 16-byte words,
// a field set in its storage format (kind 0 FP64, 1 FP32, 2 FP16) and a run
// of FP64 values (probe ring and DFT accumulators):
//   kFlagNonFinite  a NaN or an infinity (FP16 storage: a NaN),
//   kFlagOverflow   an infinity in FP16 storage, i.e. a value whose scaled
//                   magnitude rounded past the largest finite fp16 (65504).
// Classification works on the bit patterns (exponent field all ones).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t classify_word(uint4 w, int kind) {
  uint32_t f = 0u;
  const uint32_t u[4] = {w.x, w.y, w.z, w.w};
  if (kind == 0) {
#pragma unroll
    for (int q = 0; q < 4; q += 2)
      f |= ((u[q + 1] & 0x7ff00000u) == 0x7ff00000u) ? kFlagNonFinite : 0u;   // high word of each double
  } else if (kind == 1) {
#pragma unroll
    for (int q = 0; q < 4; ++q) f |= ((u[q] & 0x7f800000u) == 0x7f800000u) ? kFlagNonFinite : 0u;
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t b = (u[q] >> (16 * h)) & 0xffffu;
        if ((b & 0x7c00u) == 0x7c00u) f |= (b & 0x03ffu) ? kFlagNonFinite : kFlagOverflow;
      }
  }
  return f;
}

__global__ void __launch_bounds__(256)
status_scan_kernel(const uint4* __restrict__ fld, size_t nfld, int kind, const uint4* __restrict__ dbl,
                   size_t ndbl, uint32_t* __restrict__ flags) {
  uint32_t f = 0u;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < nfld; i += stride)
    f |= classify_word(fld[i], kind);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < ndbl; i += stride)
    f |= classify_word(dbl[i], 0);
  const uint64_t b0 = __ballot((f & kFlagNonFinite) != 0u);
  const uint64_t b1 = __ballot((f & kFlagOverflow) != 0u);
  if ((threadIdx.x & (kWave - 1)) == 0 && (b0 | b1))
    atomicOr(flags, (b0 ? kFlagNonFinite : 0u) | (b1 ? kFlagOverflow : 0u));
}

// Writes a saved state's header: 32 64-bit words passed by value (no host
// staging buffer has to outlive the launch).
struct StateHeader {
  int64_t w[32];
};

__global__ void state_header_kernel(StateHeader h, int64_t* __restrict__ dst) {
  if (threadIdx.x < 32) dst[threadIdx.x] = h.w[threadIdx.x];
}

}  // namespace yee
