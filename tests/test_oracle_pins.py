"""Pins of the FP64 oracle against what the mathematics fixes.

None of these compares the oracle with itself: each checks a closed form, an
invariant of the scheme, a symmetry or a brute-force enumeration written
independently of the vectorized update.  The paper defines no full-wave
solver and prints no numbers for one, so there are no worked examples from
it to pin against.
"""
import numpy as np
import pytest

from oracle.yee import (C0, EPS0, MU0, COMPONENTS, CpmlParams, Probe, Simulation,
                        Source, dft_accumulate, material_coefficients, round_fp16_scaled, round_fp32,
                        time_step, yee_shape)


def _random_fields(sim, rng, scale_h=1.0 / 377.0, e=True, h=True):
    """Random E^0 / H^{-1/2} with the PEC wall samples (tangential E) left at 0."""
    nx, ny, nz = sim.nx, sim.ny, sim.nz
    out = {}
    if e:
        ex = np.zeros(yee_shape("Ex", nx, ny, nz)); ex[:, 1:ny, 1:nz] = rng.standard_normal((nx, ny - 1, nz - 1))
        ey = np.zeros(yee_shape("Ey", nx, ny, nz)); ey[1:nx, :, 1:nz] = rng.standard_normal((nx - 1, ny, nz - 1))
        ez = np.zeros(yee_shape("Ez", nx, ny, nz)); ez[1:nx, 1:ny, :] = rng.standard_normal((nx - 1, ny - 1, nz))
        out.update(Ex=ex, Ey=ey, Ez=ez)
    if h:
        for c in ("Hx", "Hy", "Hz"):
            out[c] = scale_h * rng.standard_normal(yee_shape(c, nx, ny, nz))
        # normal H on the walls is never used and stays 0 in a PEC box
        out["Hx"][0] = out["Hx"][nx] = 0.0
        out["Hy"][:, 0] = out["Hy"][:, ny] = 0.0
        out["Hz"][:, :, 0] = out["Hz"][:, :, nz] = 0.0
    sim.set_fields(**out)
    return out


# ---------------------------------------------------------------------------
# Material coefficients: the semi-implicit conduction equation they solve
# ---------------------------------------------------------------------------

def test_ca_cb_solve_semi_implicit_update():
    """eps (E' - E)/dt + sigma (E' + E)/2 = R  <=>  E' = Ca E + Cb R."""
    rng = np.random.default_rng(0)
    eps_r = rng.uniform(1, 12, 100)
    sig = rng.uniform(0, 5, 100)
    dt = 1e-12
    ca, cb = material_coefficients(eps_r, sig, dt)
    eps = EPS0 * eps_r
    e, r = rng.standard_normal(100), rng.standard_normal(100)
    e_new = ca * e + cb * r
    lhs = eps * (e_new - e) / dt + sig * (e_new + e) / 2
    np.testing.assert_allclose(lhs, r, rtol=1e-12, atol=1e-12 * np.abs(r).max())


def test_time_step_is_courant_fraction():
    # cube: dt = S dx / (c sqrt(3))
    dt = time_step(1e-3, 1e-3, 1e-3, 0.99)
    assert abs(dt - 0.99 * 1e-3 / (C0 * np.sqrt(3.0))) <= 1e-15 * dt
    assert abs(dt - 1.90657e-12) < 1e-17
    assert abs(C0 * C0 * MU0 * EPS0 - 1.0) < 1e-15


# ---------------------------------------------------------------------------
# P-A1: discrete eigenmode of a PEC box follows the closed-form recurrence
# ---------------------------------------------------------------------------

def _tm_mode(nx, ny, nz, m, n):
    i = np.arange(nx + 1)
    j = np.arange(ny + 1)
    phi2 = np.outer(np.sin(m * np.pi * i / nx), np.sin(n * np.pi * j / ny))
    return np.repeat(phi2[:, :, None], nz, axis=2)


@pytest.mark.parametrize("m,n,eps", [(1, 1, 1.0), (2, 3, 2.5), (5, 4, 1.0)])
def test_eigenmode_closed_form_lossless(m, n, eps):
    nx, ny, nz = 16, 12, 5
    dx, dy, dz = 1e-3, 1.3e-3, 0.8e-3
    sim = Simulation(nx, ny, nz, dx, dy, dz, eps_r=eps)
    phi = _tm_mode(nx, ny, nz, m, n)
    sim.set_fields(Ez=phi)
    lam = (2 / dx) ** 2 * np.sin(m * np.pi / (2 * nx)) ** 2 + (2 / dy) ** 2 * np.sin(n * np.pi / (2 * ny)) ** 2
    c = 1.0 / np.sqrt(MU0 * EPS0 * eps)
    theta = 2 * np.arcsin(c * sim.dt / 2 * np.sqrt(lam))
    for step in range(1, 301):
        sim.step()
        a = np.cos((step + 0.5) * theta) / np.cos(theta / 2)
        assert np.abs(sim.E["Ez"] - a * phi).max() <= 1e-12, step
        assert not sim.E["Ex"].any() and not sim.E["Ey"].any()


def test_eigenmode_lossy_scalar_recurrence():
    """Uniform sigma > 0: a_{n+1} = (1 + Ca - Cb dt Lam/mu0) a_n - Ca a_{n-1}.

    Ca and Cb are obtained here by solving eps(E'-E)/dt + sigma(E'+E)/2 = R
    directly, not from the oracle's formula.
    """
    nx, ny, nz = 12, 10, 3
    dx = 1e-3
    eps_r, sig = 3.0, 0.4
    sim = Simulation(nx, ny, nz, dx, eps_r=eps_r, sigma=sig)
    m, n = 2, 1
    phi = _tm_mode(nx, ny, nz, m, n)
    sim.set_fields(Ez=phi)
    dt = sim.dt
    eps = EPS0 * eps_r
    g = eps / dt + sig / 2
    ca, cb = (eps / dt - sig / 2) / g, 1.0 / g
    lam = (2 / dx) ** 2 * (np.sin(m * np.pi / (2 * nx)) ** 2 + np.sin(n * np.pi / (2 * ny)) ** 2)
    k = cb * dt * lam / MU0
    a_prev, a = 1.0, ca - k
    sim.step()
    assert np.abs(sim.E["Ez"] - a * phi).max() <= 1e-13
    for _ in range(200):
        a_prev, a = a, (1 + ca - k) * a - ca * a_prev
        sim.step()
        assert np.abs(sim.E["Ez"] - a * phi).max() <= 1e-12


# ---------------------------------------------------------------------------
# P-A2: PEC cavity resonances at the discrete mode frequencies
# ---------------------------------------------------------------------------

def _windowed_peak(y, dt, f_guess, half_width):
    n = np.arange(len(y))
    w = np.hanning(len(y))
    yw = (y - y.mean()) * w

    def mag(f):
        return -np.abs(np.sum(yw * np.exp(-2j * np.pi * f * n * dt)))

    lo, hi = f_guess - half_width, f_guess + half_width
    # coarse scan then golden section
    fs = np.linspace(lo, hi, 41)
    k = int(np.argmin([mag(f) for f in fs]))
    lo, hi = fs[max(k - 1, 0)], fs[min(k + 1, 40)]
    gr = (np.sqrt(5) - 1) / 2
    a, b = lo, hi
    c, d = b - gr * (b - a), a + gr * (b - a)
    for _ in range(60):
        if mag(c) < mag(d):
            b = d
        else:
            a = c
        c, d = b - gr * (b - a), a + gr * (b - a)
    return 0.5 * (a + b)


def test_cavity_resonances_discrete_frequencies():
    nx, ny, nz = 10, 8, 6
    dx, dy, dz = 1.0e-3, 1.2e-3, 0.9e-3
    sim = Simulation(nx, ny, nz, dx, dy, dz)
    dt = sim.dt
    sim.sources = [Source(2, 3, 3, 2, "gauss_deriv", 1.0, 20 * dt, 5 * dt)]
    sim.probes = [Probe(2, 7, 5, 1)]
    sim.series = [[]]
    sim.dft = [np.zeros(0, complex)]
    nsteps = 1 << 13
    sim.run(nsteps)
    y = sim.series_array()[200:, 0]
    # discrete TM-to-z mode frequencies seen by an Ez probe (m, n >= 1, p >= 0)
    modes = []
    for m in range(1, nx):
        for n in range(1, ny):
            for p in range(0, nz):
                s = (np.sin(m * np.pi / (2 * nx)) / dx) ** 2 + (np.sin(n * np.pi / (2 * ny)) / dy) ** 2 \
                    + (np.sin(p * np.pi / (2 * nz)) / dz) ** 2
                modes.append(np.arcsin(C0 * dt * np.sqrt(s)) / (np.pi * dt))
    modes = np.sort(np.array(modes))
    bin_w = 1.0 / (len(y) * dt)
    checked = 0
    for f in modes[:12]:
        if np.min(np.abs(np.delete(modes, np.argmin(np.abs(modes - f))) - f)) < 8 * bin_w:
            continue   # not isolated enough for a window-limited estimate
        f_est = _windowed_peak(y, dt, f, 1.5 * bin_w)
        assert abs(f_est - f) / f <= 1e-4, (f, f_est)
        checked += 1
    assert checked >= 3


# ---------------------------------------------------------------------------
# P-A3: discrete energy of a closed lossless box is conserved; loss decreases it
# ---------------------------------------------------------------------------

def _energy_series(sim, nsteps):
    ws = []
    for _ in range(nsteps):
        e_n = {c: v.copy() for c, v in sim.E.items()}
        h_prev = {c: v.copy() for c, v in sim.H.items()}
        sim.step()
        ws.append(sim.energy(e_n, h_prev, sim.H))
    return np.array(ws)


def test_energy_conserved_lossless_inhomogeneous():
    rng = np.random.default_rng(3)
    nx, ny, nz = 10, 9, 8
    eps = rng.uniform(1, 5, (nx, ny, nz))
    sim = Simulation(nx, ny, nz, 1e-3, 1.1e-3, 0.9e-3, eps_r=eps)
    _random_fields(sim, rng)
    w = _energy_series(sim, 1000)
    assert np.abs(w - w[0]).max() / w[0] <= 1e-12


def test_energy_nonincreasing_lossy():
    rng = np.random.default_rng(4)
    nx, ny, nz = 8, 8, 8
    sim = Simulation(nx, ny, nz, 1e-3, eps_r=rng.uniform(1, 4, (nx, ny, nz)),
                     sigma=rng.uniform(0, 2.0, (nx, ny, nz)))
    _random_fields(sim, rng)
    w = _energy_series(sim, 300)
    assert np.all(np.diff(w) <= 1e-14 * w[0])
    assert w[-1] < 0.5 * w[0]


# ---------------------------------------------------------------------------
# P-A4: discrete Gauss law
# ---------------------------------------------------------------------------

def _div_eps_e(sim):
    nx, ny, nz = sim.nx, sim.ny, sim.nz
    def eps_of(c):
        shp = sim.E[c].shape
        ii = np.minimum(np.arange(shp[0]), nx - 1)
        jj = np.minimum(np.arange(shp[1]), ny - 1)
        kk = np.minimum(np.arange(shp[2]), nz - 1)
        return EPS0 * sim.eps_cell[np.ix_(ii, jj, kk)]
    dx_ = eps_of("Ex") * sim.E["Ex"]
    dy_ = eps_of("Ey") * sim.E["Ey"]
    dz_ = eps_of("Ez") * sim.E["Ez"]
    # interior nodes (i, j, k) in [1, n-1]^3
    return ((dx_[1:nx, 1:ny, 1:nz] - dx_[0:nx - 1, 1:ny, 1:nz]) / sim.dx
            + (dy_[1:nx, 1:ny, 1:nz] - dy_[1:nx, 0:ny - 1, 1:nz]) / sim.dy
            + (dz_[1:nx, 1:ny, 1:nz] - dz_[1:nx, 1:ny, 0:nz - 1]) / sim.dz)


def test_gauss_law_with_source():
    rng = np.random.default_rng(5)
    nx, ny, nz = 9, 8, 10
    sim = Simulation(nx, ny, nz, 1e-3, eps_r=rng.uniform(1, 6, (nx, ny, nz)))
    dt = sim.dt
    si, sj, sk = 4, 3, 5
    sim.sources = [Source(2, si, sj, sk, "gauss_deriv", 1.0, 20 * dt, 6 * dt)]
    _random_fields(sim, rng, h=False)
    d0 = _div_eps_e(sim)
    scale = np.abs(d0).max()
    touched = np.zeros_like(d0, dtype=bool)
    # the source edge Ez[si,sj,sk] joins nodes (si,sj,sk) and (si,sj,sk+1)
    touched[si - 1, sj - 1, sk - 1] = True
    touched[si - 1, sj - 1, sk] = True
    for _ in range(150):
        sim.step()
        d = _div_eps_e(sim)
        assert np.abs(d - d0)[~touched].max() <= 1e-12 * scale
    assert np.abs(d - d0)[touched].max() > 1e-6 * scale   # the source does inject charge
    # div(mu H) at cell centres stays 0 (H^{-1/2} = 0)
    H = sim.H
    divh = ((H["Hx"][1:] - H["Hx"][:-1]) / sim.dx + (H["Hy"][:, 1:] - H["Hy"][:, :-1]) / sim.dy
            + (H["Hz"][:, :, 1:] - H["Hz"][:, :, :-1]) / sim.dz)
    hscale = max(np.abs(H[c]).max() for c in H) / sim.dx
    assert np.abs(divh).max() <= 1e-12 * hscale


# ---------------------------------------------------------------------------
# P-A5: brute force on tiny grids
# ---------------------------------------------------------------------------

def _enumerate_curls(nx, ny, nz, dx, dy, dz):
    """Sparse curl operators built by visiting every sample.

    Ce maps E (all samples, concatenated Ex|Ey|Ez) to curl E at every H sample;
    Ch maps H to curl H at every E sample that is not a PEC wall sample.
    """
    def index(shapes):
        offs, tot = {}, 0
        for c, s in shapes:
            offs[c] = tot
            tot += int(np.prod(s))
        return offs, tot
    es = [(c, yee_shape(c, nx, ny, nz)) for c in ("Ex", "Ey", "Ez")]
    hs = [(c, yee_shape(c, nx, ny, nz)) for c in ("Hx", "Hy", "Hz")]
    eo, ne = index(es)
    ho, nh = index(hs)
    eshp, hshp = dict(es), dict(hs)

    def eid(c, i, j, k):
        s = eshp[c]
        if not (0 <= i < s[0] and 0 <= j < s[1] and 0 <= k < s[2]):
            return None
        return eo[c] + (i * s[1] + j) * s[2] + k

    def hid(c, i, j, k):
        s = hshp[c]
        if not (0 <= i < s[0] and 0 <= j < s[1] and 0 <= k < s[2]):
            return None
        return ho[c] + (i * s[1] + j) * s[2] + k

    Ce = np.zeros((nh, ne))
    for c, s in hs:
        for i in range(s[0]):
            for j in range(s[1]):
                for k in range(s[2]):
                    r = hid(c, i, j, k)
                    if c == "Hx":    # dEz/dy - dEy/dz at (i, j+1/2, k+1/2)
                        terms = [("Ez", i, j + 1, k, 1 / dy), ("Ez", i, j, k, -1 / dy),
                                 ("Ey", i, j, k + 1, -1 / dz), ("Ey", i, j, k, 1 / dz)]
                    elif c == "Hy":  # dEx/dz - dEz/dx at (i+1/2, j, k+1/2)
                        terms = [("Ex", i, j, k + 1, 1 / dz), ("Ex", i, j, k, -1 / dz),
                                 ("Ez", i + 1, j, k, -1 / dx), ("Ez", i, j, k, 1 / dx)]
                    else:            # dEy/dx - dEx/dy at (i+1/2, j+1/2, k)
                        terms = [("Ey", i + 1, j, k, 1 / dx), ("Ey", i, j, k, -1 / dx),
                                 ("Ex", i, j + 1, k, -1 / dy), ("Ex", i, j, k, 1 / dy)]
                    for (ec, a, b, cc, w) in terms:
                        col = eid(ec, a, b, cc)
                        assert col is not None
                        Ce[r, col] += w
    Ch = np.zeros((ne, nh))
    interior = np.zeros(ne, dtype=bool)
    for c, s in es:
        for i in range(s[0]):
            for j in range(s[1]):
                for k in range(s[2]):
                    r = eid(c, i, j, k)
                    if c == "Ex":
                        if j in (0, ny) or k in (0, nz):
                            continue
                        terms = [("Hz", i, j, k, 1 / dy), ("Hz", i, j - 1, k, -1 / dy),
                                 ("Hy", i, j, k, -1 / dz), ("Hy", i, j, k - 1, 1 / dz)]
                    elif c == "Ey":
                        if i in (0, nx) or k in (0, nz):
                            continue
                        terms = [("Hx", i, j, k, 1 / dz), ("Hx", i, j, k - 1, -1 / dz),
                                 ("Hz", i, j, k, -1 / dx), ("Hz", i - 1, j, k, 1 / dx)]
                    else:
                        if i in (0, nx) or j in (0, ny):
                            continue
                        terms = [("Hy", i, j, k, 1 / dx), ("Hy", i - 1, j, k, -1 / dx),
                                 ("Hx", i, j, k, -1 / dy), ("Hx", i, j - 1, k, 1 / dy)]
                    interior[r] = True
                    for (hc, a, b, cc, w) in terms:
                        col = hid(hc, a, b, cc)
                        assert col is not None
                        Ch[r, col] += w
    return Ce, Ch, interior, eo, ho


def test_curl_matrices_are_transposes():
    nx, ny, nz = 4, 3, 5
    Ce, Ch, interior, _, _ = _enumerate_curls(nx, ny, nz, 1.0, 1.0, 1.0)
    np.testing.assert_array_equal(Ch[interior], Ce.T[interior])
    assert not Ch[~interior].any()


def test_oracle_step_equals_matrix_step():
    rng = np.random.default_rng(6)
    nx, ny, nz = 4, 3, 5
    dx, dy, dz = 1e-3, 1.2e-3, 0.7e-3
    eps = rng.uniform(1, 4, (nx, ny, nz))
    sim = Simulation(nx, ny, nz, dx, dy, dz, eps_r=eps)
    f0 = _random_fields(sim, rng)
    Ce, Ch, interior, eo, ho = _enumerate_curls(nx, ny, nz, dx, dy, dz)
    e = np.concatenate([f0[c].ravel() for c in ("Ex", "Ey", "Ez")])
    h = np.concatenate([f0[c].ravel() for c in ("Hx", "Hy", "Hz")])
    # per-E-sample eps by the staircase rule, enumerated
    epsv = np.empty_like(e)
    for c in ("Ex", "Ey", "Ez"):
        s = yee_shape(c, nx, ny, nz)
        for i in range(s[0]):
            for j in range(s[1]):
                for k in range(s[2]):
                    epsv[eo[c] + (i * s[1] + j) * s[2] + k] = eps[min(i, nx - 1), min(j, ny - 1), min(k, nz - 1)]
    for _ in range(3):
        h = h - sim.dt / MU0 * (Ce @ e)
        e = np.where(interior, e + sim.dt / (EPS0 * epsv) * (Ch @ h), e)
        sim.step()
    e_or = np.concatenate([sim.E[c].ravel() for c in ("Ex", "Ey", "Ez")])
    h_or = np.concatenate([sim.H[c].ravel() for c in ("Hx", "Hy", "Hz")])
    np.testing.assert_allclose(e_or, e, rtol=0, atol=1e-13 * np.abs(e).max())
    np.testing.assert_allclose(h_or, h, rtol=0, atol=1e-13 * np.abs(h).max())


def _loop_step(st, nx, ny, nz, d, dt, ca, cb, prof, src_val, src):
    """One step written sample by sample (CPML included), for tiny grids.

    prof[(side, axis)] = (b, a, 1/kappa) indexed by the integer sample index
    along that axis (side "E": position i; side "H": position i + 1/2).
    """
    E, H, P = st["E"], st["H"], st["P"]
    dx, dy, dz = d
    Hn = {c: H[c].copy() for c in H}

    def cp(side, ax, idx, key, diff):
        b, a, ki = prof[(side, ax)]
        P[key][idx] = b[idx[ "xyz".index(ax)]] * P[key][idx] + a[idx["xyz".index(ax)]] * diff
        return ki[idx["xyz".index(ax)]] * diff + P[key][idx]

    for (i, j, k), _ in np.ndenumerate(H["Hx"]):
        t1 = cp("H", "y", (i, j, k), "Hxy", (E["Ez"][i, j + 1, k] - E["Ez"][i, j, k]) / dy)
        t2 = cp("H", "z", (i, j, k), "Hxz", (E["Ey"][i, j, k + 1] - E["Ey"][i, j, k]) / dz)
        Hn["Hx"][i, j, k] = H["Hx"][i, j, k] - dt / MU0 * (t1 - t2)
    for (i, j, k), _ in np.ndenumerate(H["Hy"]):
        t1 = cp("H", "z", (i, j, k), "Hyz", (E["Ex"][i, j, k + 1] - E["Ex"][i, j, k]) / dz)
        t2 = cp("H", "x", (i, j, k), "Hyx", (E["Ez"][i + 1, j, k] - E["Ez"][i, j, k]) / dx)
        Hn["Hy"][i, j, k] = H["Hy"][i, j, k] - dt / MU0 * (t1 - t2)
    for (i, j, k), _ in np.ndenumerate(H["Hz"]):
        t1 = cp("H", "x", (i, j, k), "Hzx", (E["Ey"][i + 1, j, k] - E["Ey"][i, j, k]) / dx)
        t2 = cp("H", "y", (i, j, k), "Hzy", (E["Ex"][i, j + 1, k] - E["Ex"][i, j, k]) / dy)
        Hn["Hz"][i, j, k] = H["Hz"][i, j, k] - dt / MU0 * (t1 - t2)
    H.update(Hn)
    En = {c: E[c].copy() for c in E}
    for (i, j, k), _ in np.ndenumerate(E["Ex"]):
        if j in (0, ny) or k in (0, nz):
            continue
        t1 = cp("E", "y", (i, j, k), "Exy", (H["Hz"][i, j, k] - H["Hz"][i, j - 1, k]) / dy)
        t2 = cp("E", "z", (i, j, k), "Exz", (H["Hy"][i, j, k] - H["Hy"][i, j, k - 1]) / dz)
        cell = (min(i, nx - 1), min(j, ny - 1), min(k, nz - 1))
        En["Ex"][i, j, k] = ca[cell] * E["Ex"][i, j, k] + cb[cell] * (t1 - t2)
    for (i, j, k), _ in np.ndenumerate(E["Ey"]):
        if i in (0, nx) or k in (0, nz):
            continue
        t1 = cp("E", "z", (i, j, k), "Eyz", (H["Hx"][i, j, k] - H["Hx"][i, j, k - 1]) / dz)
        t2 = cp("E", "x", (i, j, k), "Eyx", (H["Hz"][i, j, k] - H["Hz"][i - 1, j, k]) / dx)
        cell = (min(i, nx - 1), min(j, ny - 1), min(k, nz - 1))
        En["Ey"][i, j, k] = ca[cell] * E["Ey"][i, j, k] + cb[cell] * (t1 - t2)
    for (i, j, k), _ in np.ndenumerate(E["Ez"]):
        if i in (0, nx) or j in (0, ny):
            continue
        t1 = cp("E", "x", (i, j, k), "Ezx", (H["Hy"][i, j, k] - H["Hy"][i - 1, j, k]) / dx)
        t2 = cp("E", "y", (i, j, k), "Ezy", (H["Hx"][i, j, k] - H["Hx"][i, j - 1, k]) / dy)
        cell = (min(i, nx - 1), min(j, ny - 1), min(k, nz - 1))
        En["Ez"][i, j, k] = ca[cell] * E["Ez"][i, j, k] + cb[cell] * (t1 - t2)
    En["Ez"][src] += src_val
    E.update(En)


def _loop_profile(n, L, dw, dt, half, m=3.0, kappa_max=2.0, alpha_max=0.0):
    """(b, a, 1/kappa) per sample index, from the layer's depth written per sample."""
    cnt = n if half else n + 1
    b, a, ki = np.ones(cnt), np.zeros(cnt), np.ones(cnt)
    smax = 0.8 * (m + 1) / (np.sqrt(MU0 / EPS0) * dw)
    for idx in range(cnt):
        pos = idx + (0.5 if half else 0.0)
        if pos < L:
            x = (L - pos) / L
        elif pos > n - L:
            x = (pos - (n - L)) / L
        else:
            continue
        sig = smax * x ** m
        kap = 1 + (kappa_max - 1) * x ** m
        alp = alpha_max * (1 - x)
        b[idx] = np.exp(-(sig / kap + alp) * dt / EPS0)
        a[idx] = sig * (b[idx] - 1) / (kap * (sig + kap * alp))
        ki[idx] = 1 / kap
    return b, a, ki


def test_oracle_matches_per_sample_loops_with_cpml():
    rng = np.random.default_rng(7)
    nx, ny, nz = 6, 5, 7
    dx, dy, dz = 1e-3, 1.1e-3, 0.9e-3
    L = (2, 2, 3)
    alpha_max = 0.05
    eps = rng.uniform(1, 4, (nx, ny, nz))
    sig = rng.uniform(0, 0.5, (nx, ny, nz))
    cp = CpmlParams(cells=L, m=3.0, kappa_max=2.0, alpha_max=alpha_max)
    sim = Simulation(nx, ny, nz, dx, dy, dz, eps_r=eps, sigma=sig, cpml=cp)
    dt = sim.dt
    src = Source(2, 3, 2, 3, "mod_gauss", 2.0, 3 * dt, 2 * dt, 30e9)
    sim.sources = [src]
    f0 = _random_fields(sim, rng)
    eps_abs = EPS0 * eps
    s = sig * dt / (2 * eps_abs)
    ca = (1 - s) / (1 + s)
    cb = dt / eps_abs / (1 + s)
    prof = {}
    for ax, n, dw, l in zip("xyz", (nx, ny, nz), (dx, dy, dz), L):
        prof[("E", ax)] = _loop_profile(n, l, dw, dt, False, kappa_max=2.0, alpha_max=alpha_max)
        prof[("H", ax)] = _loop_profile(n, l, dw, dt, True, kappa_max=2.0, alpha_max=alpha_max)
    st = {"E": {c: f0[c].copy() for c in ("Ex", "Ey", "Ez")},
          "H": {c: f0[c].copy() for c in ("Hx", "Hy", "Hz")},
          "P": {"Hxy": np.zeros(yee_shape("Hx", nx, ny, nz)), "Hxz": np.zeros(yee_shape("Hx", nx, ny, nz)),
                "Hyz": np.zeros(yee_shape("Hy", nx, ny, nz)), "Hyx": np.zeros(yee_shape("Hy", nx, ny, nz)),
                "Hzx": np.zeros(yee_shape("Hz", nx, ny, nz)), "Hzy": np.zeros(yee_shape("Hz", nx, ny, nz)),
                "Exy": np.zeros(yee_shape("Ex", nx, ny, nz)), "Exz": np.zeros(yee_shape("Ex", nx, ny, nz)),
                "Eyz": np.zeros(yee_shape("Ey", nx, ny, nz)), "Eyx": np.zeros(yee_shape("Ey", nx, ny, nz)),
                "Ezx": np.zeros(yee_shape("Ez", nx, ny, nz)), "Ezy": np.zeros(yee_shape("Ez", nx, ny, nz))}}
    for n in range(4):
        u = ((n + 1) * dt - src.t0) / src.tau
        w = np.sin(2 * np.pi * src.f0 * ((n + 1) * dt - src.t0)) * np.exp(-u * u)
        _loop_step(st, nx, ny, nz, (dx, dy, dz), dt, ca, cb, prof, src.amp * w, (src.i, src.j, src.k))
        sim.step()
    for c in ("Ex", "Ey", "Ez"):
        np.testing.assert_allclose(sim.E[c], st["E"][c], rtol=0, atol=1e-13 * np.abs(st["E"][c]).max())
    for c in ("Hx", "Hy", "Hz"):
        np.testing.assert_allclose(sim.H[c], st["H"][c], rtol=0, atol=1e-13 * np.abs(st["H"][c]).max())
    # the psi arrays agree on their common (interior) samples
    sl = {"Ex": (slice(None), slice(1, ny), slice(1, nz)), "Ey": (slice(1, nx), slice(None), slice(1, nz)),
          "Ez": (slice(1, nx), slice(1, ny), slice(None))}
    for key in ("Exy", "Exz", "Eyz", "Eyx", "Ezx", "Ezy"):
        ref = st["P"][key][sl["E" + key[1]]]
        np.testing.assert_allclose(sim.psi[key], ref, rtol=0, atol=1e-13 * max(np.abs(ref).max(), 1e-300))
        assert np.abs(ref).max() > 0
    for key in ("Hxy", "Hxz", "Hyz", "Hyx", "Hzx", "Hzy"):
        ref = st["P"][key]
        np.testing.assert_allclose(sim.psi[key], ref, rtol=0, atol=1e-13 * np.abs(ref).max())


# ---------------------------------------------------------------------------
# P-A6: CPML
# ---------------------------------------------------------------------------

def test_cpml_with_zero_conductivity_is_the_pec_box():
    rng = np.random.default_rng(8)
    nx, ny, nz = 12, 10, 9
    kw = dict(eps_r=rng.uniform(1, 3, (nx, ny, nz)))
    a = Simulation(nx, ny, nz, 1e-3, cpml=CpmlParams(cells=3, sigma_max=0.0, kappa_max=1.0, alpha_max=0.0), **kw)
    b = Simulation(nx, ny, nz, 1e-3, **kw)
    f = _random_fields(a, rng)
    b.set_fields(**f)
    a.run(20)
    b.run(20)
    for c in COMPONENTS:
        np.testing.assert_array_equal(a.component(c), b.component(c))


def _plate_run(n, L, steps, src_off, probe_off):
    """Parallel-plate (PEC in z, 2 cells) TEM propagation in x-y with a CPML of L cells."""
    c = n // 2
    sim = Simulation(n, n, 2, 1e-3, cpml=CpmlParams(cells=(L, L, 0)))
    dt = sim.dt
    sim.sources = [Source(2, c + src_off, c, 0, "gauss_deriv", 1.0, 30 * dt, 8 * dt)]
    sim.probes = [Probe(2, c + probe_off, c, 0)]
    sim.series = [[]]
    sim.dft = [np.zeros(0, complex)]
    sim.run(steps)
    return sim.series_array()[:, 0]


def test_cpml_reflection_small():
    n, L, steps = 40, 10, 260
    # probe 5 cells in front of the layer (layer starts at n-L)
    probe_off = (n - L - 5) - n // 2
    y = _plate_run(n, L, steps, 0, probe_off)
    big = n + 2 * 70       # no wall echo reaches the probe within `steps`
    y_ref = _plate_run(big, 0, steps, 0, probe_off)
    err = np.abs(y - y_ref).max() / np.abs(y_ref).max()
    assert err < 10 ** (-60 / 20), err    # calibrated: about -93 dB
    # without the layer the same grid reflects at O(1)
    y_pec = _plate_run(n, 0, steps, 0, probe_off)
    assert np.abs(y_pec - y_ref).max() / np.abs(y_ref).max() > 0.3


# ---------------------------------------------------------------------------
# P-A7: mirror symmetry (checks the half-cell offsets, CPML included)
# ---------------------------------------------------------------------------

def test_mirror_symmetry_with_cpml():
    nx, ny, nz = 16, 14, 13
    sim = Simulation(nx, ny, nz, 1e-3, eps_r=2.2, sigma=0.01, cpml=CpmlParams(cells=(4, 3, 4), kappa_max=1.5,
                                                                               alpha_max=0.02))
    dt = sim.dt
    sim.sources = [Source(2, nx // 2, ny // 2, (nz - 1) // 2, "gauss_deriv", 1.0, 20 * dt, 6 * dt)]
    sim.run(60)
    E, H = sim.E, sim.H
    tol = 1e-13
    def chk(a, b, sign):
        assert np.abs(a - sign * b).max() <= tol * max(np.abs(a).max(), 1e-300)
    # x mirror: i -> nx - i at integer positions, i -> nx-1-i at half positions
    chk(E["Ez"], E["Ez"][::-1], 1); chk(E["Ey"], E["Ey"][::-1], 1); chk(E["Ex"], E["Ex"][::-1], -1)
    chk(H["Hx"], H["Hx"][::-1], 1); chk(H["Hy"], H["Hy"][::-1], -1); chk(H["Hz"], H["Hz"][::-1], -1)
    # y mirror
    chk(E["Ez"], E["Ez"][:, ::-1], 1); chk(E["Ex"], E["Ex"][:, ::-1], 1); chk(E["Ey"], E["Ey"][:, ::-1], -1)
    chk(H["Hy"], H["Hy"][:, ::-1], 1); chk(H["Hx"], H["Hx"][:, ::-1], -1); chk(H["Hz"], H["Hz"][:, ::-1], -1)
    # z mirror (source edge centred): Ez even, Ex/Ey odd, Hx/Hy even, Hz odd
    chk(E["Ez"], E["Ez"][:, :, ::-1], 1); chk(E["Ex"], E["Ex"][:, :, ::-1], -1); chk(E["Ey"], E["Ey"][:, :, ::-1], -1)
    chk(H["Hx"], H["Hx"][:, :, ::-1], 1); chk(H["Hy"], H["Hy"][:, :, ::-1], 1); chk(H["Hz"], H["Hz"][:, :, ::-1], -1)
    assert np.abs(E["Ex"]).max() > 0 and np.abs(H["Hz"]).max() >= 0


# ---------------------------------------------------------------------------
# P-A8: running DFT against the geometric-series closed form
# ---------------------------------------------------------------------------

def test_running_dft_geometric_series():
    dt = 0.953287e-12
    fa = 7.3e9
    freqs = 10e9 * (0.5 + np.arange(64) / 63.0)
    N = 1000
    acc = np.zeros(64, complex)
    for n in range(1, N + 1):
        acc = dft_accumulate(acc, np.cos(2 * np.pi * fa * n * dt), n, freqs, dt)
    a = 2 * np.pi * fa * dt
    b = 2 * np.pi * freqs * dt

    def geo(r):
        return r * (1 - r ** N) / (1 - r)
    closed = 0.5 * dt * (geo(np.exp(1j * (a - b))) + geo(np.exp(-1j * (a + b))))
    np.testing.assert_allclose(acc, closed, rtol=0, atol=1e-13 * np.abs(closed).max())


# ---------------------------------------------------------------------------
# Source waveforms and FP16 storage rounding
# ---------------------------------------------------------------------------

def test_waveform_closed_forms():
    s = Source(2, 0, 0, 0, "gauss_deriv", 1.0, 40.0, 12.0)
    t_peak = 40.0 - 12.0 / np.sqrt(2.0)
    assert abs(s.waveform(t_peak) - np.sqrt(2.0 / np.e)) < 1e-15
    assert s.waveform(40.0) == 0.0
    t = np.linspace(0, 80, 200001)
    assert abs(np.trapezoid(s.waveform(t), t)) < 1e-3    # net injected charge ~ 0
    m = Source(2, 0, 0, 0, "mod_gauss", 1.0, 200e-12, 50e-12, 10e9)
    assert m.waveform(200e-12) == 0.0
    assert abs(m.waveform(200e-12 + 25e-12) - np.exp(-0.25)) < 1e-15


def test_fp32_rounding_rules():
    assert round_fp32(1 + 2.0 ** -24) == 1.0                         # tie -> even
    assert round_fp32(1 + 3 * 2.0 ** -24) == 1 + 2.0 ** -22           # tie -> even (up)
    assert round_fp32(2.0 ** -149) == 2.0 ** -149                     # smallest subnormal kept
    assert round_fp32(2.0 ** -151) == 0.0
    x = np.random.default_rng(1).standard_normal(1000)
    assert np.all(np.abs(round_fp32(x) - x) <= 2.0 ** -24 * np.abs(x))


def test_fp16_rounding_rules():
    assert round_fp16_scaled(1 + 2.0 ** -11, 0) == 1.0              # tie -> even
    assert round_fp16_scaled(1 + 3 * 2.0 ** -11, 0) == 1 + 2.0 ** -9  # tie -> even (up)
    assert round_fp16_scaled(2.0 ** -24, 0) == 2.0 ** -24            # smallest subnormal kept
    assert round_fp16_scaled(2.0 ** -26, 0) == 0.0
    assert np.isinf(round_fp16_scaled(70000.0, 0))
    x = np.random.default_rng(0).standard_normal(1000) / 377.0
    r = round_fp16_scaled(x, 9)
    assert np.all(np.abs(r - x) <= 2.0 ** -11 * np.abs(x) + 2.0 ** -25 * 2.0 ** -9)
    assert round_fp16_scaled(3.0 * 2.0 ** -9, 9) == 3.0 * 2.0 ** -9   # exact scale


# ---------------------------------------------------------------------------
# FP32 arithmetic mode: the same step in float32
# ---------------------------------------------------------------------------

def _lossy_cpml_pair(storage, fp16_exp=(0, 0, 0, 9, 9, 9)):
    rng = np.random.default_rng(11)
    nx, ny, nz = 14, 12, 16
    eps = rng.uniform(1, 6, (nx, ny, nz))
    sig = rng.uniform(0, 0.3, (nx, ny, nz))
    cp = CpmlParams(cells=(3, 3, 4), m=3.0, kappa_max=3.0, alpha_max=0.05)
    sims = []
    for arith in ("f64", "f32"):
        sim = Simulation(nx, ny, nz, 1e-3, eps_r=eps, sigma=sig, cpml=cp, storage=storage if arith == "f32" else "f64",
                         fp16_exp=fp16_exp, arith=arith)
        sim.sources = [Source(2, 7, 6, 8, "mod_gauss", 1.0, 8 * sim.dt, 3 * sim.dt, 40e9)]
        sim.probes = [Probe(2, 5, 4, 6, np.array([30e9, 45e9]))]
        sim.series, sim.dft = [[]], [np.zeros(2, complex)]
        _random_fields(sim, np.random.default_rng(5), scale_h=1.0 / 377.0)
        sims.append(sim)
    return sims


def test_fp32_arithmetic_follows_the_fp64_step():
    """arith="f32": every array stays float32 (no operation widens it), and 60
    steps of a lossy grid with CPML in all three axes, a source and a probe
    agree with the FP64 oracle to FP32 accuracy: each component and psi
    array to 1e-5 relative L2 (one step rounds at 2^-24; the growth over 60
    steps stays far below 1e-5), the probe series and DFT too.  A term
    computed in FP64 or dropped would break the dtype or the agreement."""
    s64, s32 = _lossy_cpml_pair("f64")
    for _ in range(60):
        s64.step()
        s32.step()
    for c in COMPONENTS:
        a32, a64 = s32.component(c), s64.component(c)
        assert a32.dtype == np.float32, c
        assert np.linalg.norm(a32 - a64) <= 1e-5 * np.linalg.norm(a64), c
    for k in s64.psi:
        assert s32.psi[k].dtype == np.float32, k
        n = np.linalg.norm(s64.psi[k])
        assert np.linalg.norm(s32.psi[k] - s64.psi[k]) <= 1e-5 * n + 1e-30, k
    a, b = s32.series_array(), s64.series_array()
    assert np.linalg.norm(a - b) <= 1e-5 * np.linalg.norm(b)
    assert np.linalg.norm(s32.dft[0] - s64.dft[0]) <= 1e-5 * np.linalg.norm(s64.dft[0])


def test_fp16_storage_with_fp32_arithmetic_stores_fp16_values():
    """storage="f16" with arith="f32": every stored field value times 2^s is
    an fp16 number (the rounding happens on the FP32 result), the psi arrays
    stay unrounded float32, and the run tracks FP64 within the fp16 storage
    error (2^-11 relative per value)."""
    exps = (4, 4, 4, 12, 12, 12)
    s64, s16 = _lossy_cpml_pair("f16", fp16_exp=exps)
    for _ in range(30):
        s64.step()
        s16.step()
    for ci, c in enumerate(COMPONENTS):
        x = s16.component(c).astype(np.float64) * 2.0 ** exps[ci]
        assert np.array_equal(x.astype(np.float16).astype(np.float64), x), c
        a64 = s64.component(c)
        assert np.linalg.norm(s16.component(c) - a64) <= 4e-3 * np.linalg.norm(a64), c   # measured 1.1e-3 to 1.3e-3
    assert any(not np.array_equal(v.astype(np.float16).astype(np.float32), v)
               for v in s16.psi.values() if np.any(v))
