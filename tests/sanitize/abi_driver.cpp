// Host-side driver of the two C ABIs for the sanitizer build: it runs every
// host path that needs no device (configuration, validation, workspace
// sizing, the FP64 S-parameter combination, the argument checks of the
// device entry points) so that AddressSanitizer and UndefinedBehaviorSanitizer
// see the host code of libyee and libraymeta.  Built by
// tests/test_host_sanitizers.py with the runtimes compiled host-only; it
// never launches a kernel.  Exit status: number of failed checks.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "raymeta.h"
#include "yee.h"

static int g_fail = 0;

#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++g_fail;                                                            \
    }                                                                      \
  } while (0)

static yee_grid_desc desc(int nx, int ny, int nz, int precision, int cpml) {
  yee_grid_desc d;
  std::memset(&d, 0, sizeof d);
  d.nx = nx; d.ny = ny; d.nz = nz;
  d.dx = d.dy = d.dz = 1e-3;
  d.courant = 0.99;
  d.precision = precision;
  for (int q = 0; q < 3; ++q) d.cpml_cells[q] = cpml;
  d.cpml_m = 3.0;
  d.cpml_sigma_max = -1.0;
  d.cpml_kappa_max = 1.5;
  d.cpml_alpha_max = 0.02;
  for (int q = 0; q < 6; ++q) d.fp16_exp[q] = q < 3 ? 12 : 21;
  d.series_len = 16;
  return d;
}

static void yee_paths() {
  CHECK(yee_api_version() == YEE_API_VERSION);
  yee_ctx* c = nullptr;
  // invalid descriptions
  yee_grid_desc bad = desc(16, 16, 16, YEE_F32, 0);
  bad.courant = 1.5;
  CHECK(yee_create(&bad, &c) == YEE_EINVAL && c == nullptr);
  CHECK(std::strlen(yee_last_error()) > 0);
  bad = desc(16, 16, 16, YEE_F32, 9);
  CHECK(yee_create(&bad, &c) == YEE_EINVAL);
  bad = desc(1, 16, 16, YEE_F32, 0);
  CHECK(yee_create(&bad, &c) == YEE_EINVAL);
  bad = desc(16, 16, 16, 7, 0);
  CHECK(yee_create(&bad, &c) == YEE_EINVAL);
  bad = desc(16, 16, 16, YEE_F32, 0);
  bad.series_len = 0;
  CHECK(yee_create(&bad, &c) == YEE_EINVAL);
  CHECK(yee_create(nullptr, &c) == YEE_EINVAL);

  for (int prec : {YEE_F64, YEE_F32, YEE_F16S}) {
    const int nx = 37, ny = 29, nz = 23;
    yee_grid_desc d = desc(nx, ny, nz, prec, 4);
    CHECK(yee_create(&d, &c) == YEE_OK && c != nullptr);
    double dt = 0.0;
    CHECK(yee_time_step(c, &dt) == YEE_OK && dt > 0.0);
    // materials: a 3 x 2 x 2 block lattice
    std::vector<int32_t> sx(nx), sy(ny), sz(nz);
    for (int i = 0; i < nx; ++i) sx[i] = i * 3 / nx;
    for (int j = 0; j < ny; ++j) sy[j] = j * 2 / ny;
    for (int k = 0; k < nz; ++k) sz[k] = k * 2 / nz;
    std::vector<double> eps(12, 2.0), sig(12, 0.01);
    CHECK(yee_set_materials(c, 3, 2, 2, sx.data(), sy.data(), sz.data(), eps.data(), sig.data()) == YEE_OK);
    eps[5] = 0.0;
    CHECK(yee_set_materials(c, 3, 2, 2, sx.data(), sy.data(), sz.data(), eps.data(), sig.data()) == YEE_EINVAL);
    eps[5] = 2.0;
    sx[4] = 3;   // segment beyond nsx
    CHECK(yee_set_materials(c, 3, 2, 2, sx.data(), sy.data(), sz.data(), eps.data(), sig.data()) == YEE_EINVAL);
    sx[4] = 0;
    // PEC masks: planes (merged) and a volume mask
    std::vector<uint8_t> plane((size_t)nx * ny, 0), vol((size_t)nx * ny * nz, 0);
    plane[5 * nx + 7] = 3;
    CHECK(yee_add_pec_plane(c, 0, plane.data()) == YEE_EINVAL);
    CHECK(yee_add_pec_plane(c, 6, plane.data()) == YEE_OK);
    CHECK(yee_add_pec_plane(c, 6, plane.data()) == YEE_OK);
    vol[(size_t)(6 * ny + 3) * nx + 2] = 4;
    vol[(size_t)(0 * ny + 3) * nx + 2] = 4;
    CHECK(yee_set_pec_mask(c, vol.data()) == YEE_OK);
    vol[17] = 9;
    CHECK(yee_set_pec_mask(c, vol.data()) == YEE_EINVAL);
    // sources, probes, frequencies
    yee_source s{2, 10, 11, 12, YEE_MOD_GAUSS, 1.0, 1e-10, 5e-11, 1e10};
    CHECK(yee_add_source(c, &s) == YEE_OK);
    s.i = nx;
    CHECK(yee_add_source(c, &s) == YEE_EINVAL);
    int32_t pid = -1;
    CHECK(yee_add_probe(c, 2, 8, 9, 10, &pid) == YEE_OK && pid == 0);
    CHECK(yee_add_probe(c, 4, 8, 9, 10, &pid) == YEE_OK && pid == 1);
    CHECK(yee_add_probe(c, 6, 8, 9, 10, &pid) == YEE_EINVAL);
    const double f[3] = {5e9, 1e10, 1.5e10};
    CHECK(yee_set_dft_freqs(c, f, 3) == YEE_OK);
    int64_t fp = 0;
    CHECK(yee_footprint(c, &fp) == YEE_OK && fp > 0);
    CHECK(yee_set_launch(c, 2, 8, 1) == YEE_OK);
    CHECK(yee_set_time_blocking(c, 5, 0, 0) == YEE_EINVAL);
    // calls that need a bound workspace
    uint32_t flags = 0;
    int64_t nb = 0;
    CHECK(yee_step(c, 1, nullptr) == YEE_ESTATE);
    CHECK(yee_reset(c, nullptr) == YEE_ESTATE);
    CHECK(yee_status_flags(c, &flags, nullptr) == YEE_ESTATE);
    CHECK(yee_state_bytes(c, &nb) == YEE_ESTATE);
    CHECK(yee_save_state(c, reinterpret_cast<void*>(4096), 1 << 20, nullptr) == YEE_ESTATE);
    CHECK(yee_load_state(c, reinterpret_cast<void*>(4096), 1 << 20, nullptr) == YEE_ESTATE);
    CHECK(yee_bind_workspace(c, nullptr, fp) == YEE_EINVAL);
    CHECK(yee_bind_workspace(c, reinterpret_cast<void*>(4096), fp - 256) != YEE_OK);
    int64_t stride = 0;
    int32_t pitch = 0;
    CHECK(yee_debug_layout(c, &stride, &pitch) == YEE_OK && stride > 0 && pitch >= nx);
    CHECK(yee_debug_set_write_counts(c, reinterpret_cast<uint32_t*>(4096), 1) == YEE_ENOMEM);
    // the adjoint needs a bound context; the batch a bound workspace
    const int32_t box[6] = {4, 10, 4, 10, 4, 10};
    yee_adjoint* adj = nullptr;
    CHECK(yee_adjoint_create(c, 20, 4, box, &adj) != YEE_OK && adj == nullptr);
    yee_destroy(c);
    c = nullptr;
  }
  yee_destroy(nullptr);

  // the batch descriptor table: sizing and admission before binding
  int64_t tb = 0;
  CHECK(yee_batch_footprint(8, &tb) == YEE_OK && tb > 0);
  CHECK(yee_batch_footprint(0, &tb) == YEE_EINVAL);
  yee_batch* b = nullptr;
  CHECK(yee_batch_create(8, int64_t(1) << 30, 16, &b) == YEE_OK && b != nullptr);
  CHECK(yee_batch_set_precision(b, 9) == YEE_EINVAL);
  CHECK(yee_batch_set_precision(nullptr, YEE_F32) == YEE_EINVAL);
  CHECK(yee_batch_set_precision(b, YEE_F16S) == YEE_OK);
  CHECK(yee_batch_set_precision(b, YEE_F32) == YEE_OK);
  int32_t slot = -1;
  yee_grid_desc d = desc(32, 32, 32, YEE_F32, 4);
  CHECK(yee_create(&d, &c) == YEE_OK);
  CHECK(yee_batch_admit(b, c, 10, &slot) == YEE_ESTATE);
  int32_t active = -1;
  int64_t used = -1;
  CHECK(yee_batch_info(b, &active, &used) == YEE_OK && active == 0 && used == 0);
  yee_batch_destroy(b);
  yee_destroy(c);

  // S-parameters (host FP64): two ports of two probes each over 5 frequencies
  const int np = 4, nf = 5, nports = 2;
  std::vector<double> rr(np * nf), ri(np * nf), dr(np * nf), di(np * nf);
  for (int q = 0; q < np * nf; ++q) {
    rr[q] = 1.0 + 0.1 * q; ri[q] = 0.05 * q; dr[q] = 0.5 + 0.07 * q; di[q] = -0.02 * q;
  }
  const int32_t off[3] = {0, 2, 4}, probe[4] = {0, 1, 2, 3};
  const double w[4] = {1e-3, 1e-3, 1e-3, 1e-3};
  std::vector<double> vr(nports * nf), vi(nports * nf), ur(nports * nf), ui(nports * nf), sr(nports * nf),
      si(nports * nf);
  CHECK(yee_sparams(np, nf, rr.data(), ri.data(), dr.data(), di.data(), nports, off, probe, w, vr.data(), vi.data(),
                    ur.data(), ui.data(), sr.data(), si.data()) == YEE_OK);
  CHECK(std::isfinite(sr[0]) && std::isfinite(si[nports * nf - 1]));
  const int32_t bad_probe[4] = {0, 1, 2, 4};
  CHECK(yee_sparams(np, nf, rr.data(), ri.data(), dr.data(), di.data(), nports, off, bad_probe, w, nullptr, nullptr,
                    nullptr, nullptr, sr.data(), si.data()) == YEE_EINVAL);
  const int32_t bad_off[3] = {0, 3, 2};
  CHECK(yee_sparams(np, nf, rr.data(), ri.data(), dr.data(), di.data(), nports, bad_off, probe, w, nullptr, nullptr,
                    nullptr, nullptr, sr.data(), si.data()) == YEE_EINVAL);
}

static void raymeta_paths() {
  CHECK(rmd_api_version() == 2);
  const uintptr_t p = 4096;   // never dereferenced: every call below fails its checks first
  rmd_scene sc;
  std::memset(&sc, 0, sizeof sc);
  sc.n_meshes = 4; sc.n_tris = 1024; sc.n_verts = 600; sc.n_rays = 100000; sc.n_hits = 175000;
  sc.mesh_tri_off = reinterpret_cast<const int32_t*>(p);
  sc.tris = reinterpret_cast<const int32_t*>(p);
  sc.verts = reinterpret_cast<const double*>(p);
  sc.ray_off = reinterpret_cast<const int32_t*>(p);
  sc.hit_mesh = reinterpret_cast<const int32_t*>(p);
  sc.hit_tri = reinterpret_cast<const int32_t*>(p);
  sc.hit_u = reinterpret_cast<const float*>(p);
  sc.hit_v = reinterpret_cast<const float*>(p);
  rmd_radar r;
  std::memset(&r, 0, sizeof r);
  r.f_c = 77e9; r.bandwidth = 1e9; r.t_chirp = 40e-6; r.f_s = 10e6; r.n_samples = 256; r.n_chirps = 8;
  int64_t need = 0;
  CHECK(rmd_workspace_bytes(&sc, &r, 4, 8, &need) == RMD_OK && need > 0);
  CHECK(rmd_workspace_bytes(&sc, &r, 0, 8, &need) == RMD_EINVAL);
  r.n_samples = RMD_MAX_SAMPLES + 1;
  CHECK(rmd_workspace_bytes(&sc, &r, 4, 8, &need) == RMD_EINVAL);
  r.n_samples = 256;
  void* vp = reinterpret_cast<void*>(p);
  float* fp = reinterpret_cast<float*>(p);
  const double* dp = reinterpret_cast<const double*>(p);
  CHECK(rmd_if_cube(&sc, &r, 4, dp, nullptr, 0, 8, fp, vp, need - 8, nullptr) == RMD_EINVAL);
  CHECK(rmd_if_cube(&sc, &r, 4, dp, nullptr, 0, 8, fp, reinterpret_cast<void*>(p + 4), need, nullptr) == RMD_EINVAL);
  CHECK(rmd_if_cube(&sc, &r, 4, dp, nullptr, 5, 8, fp, vp, need, nullptr) == RMD_EINVAL);
  CHECK(rmd_if_cube_direct(&sc, &r, 4, nullptr, nullptr, 0, 8, fp, vp, need, nullptr) == RMD_EINVAL);
  rmd_scene big = sc;
  big.n_rays = 1 << 22;
  big.n_hits = int64_t(7) << 20;
  r.n_samples = 1024;
  r.n_chirps = 16;
  CHECK(rmd_if_cube_static(&big, &r, 16, dp, nullptr, 0, 16, fp, nullptr) == RMD_EINVAL);
  CHECK(rmd_range_doppler(fp, fp, 2, 96, 512, nullptr) == RMD_EINVAL);
  CHECK(rmd_range_doppler(fp, fp, 2, 128, 8192, nullptr) == RMD_EINVAL);
  rmd_span_rule rule{5, 1, 3};
  CHECK(rmd_span_weights(&sc, reinterpret_cast<const uint8_t*>(p), &rule, nullptr, fp, nullptr) == RMD_EINVAL);
  sc.n_rays = 0;
  CHECK(rmd_check_scene(&sc, 8, vp, &need, nullptr) == RMD_EINVAL);
  CHECK(std::strlen(rmd_last_error()) > 0);
}

int main() {
  yee_paths();
  raymeta_paths();
  std::printf("%s: %d failed checks\n", g_fail ? "FAIL" : "ok", g_fail);
  return g_fail;
}
