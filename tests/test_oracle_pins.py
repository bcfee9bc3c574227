"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test names the passage it checks.  None of them re-types the oracle's
update formulas: the expected values come from closed forms (Fourier modes,
the layer modes of Thm. 1), conserved quantities, the untruncated free-space
run (the paper's own reflection measurement, Figs. 2/3), the 1-D Courant-1
light cone, and the properties the paper states (Thm. 3, Fig. 5, Fig. 6).
"""
import json
import math
import os

import numpy as np
import pytest

import synthetic
from oracle import closed_forms as cf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _state_part(mode, part):
    import oracle
    return oracle.State(part(mode["U"]).copy(), part(mode["Uprev"]).copy(),
                        [part(p).copy() for p in mode["Phi"]],
                        [part(p).copy() for p in mode["Psi"]])


# --------------------------------------------------------------------------
# Thm. 1 (Eq. IntroSolution, IntroDecayRate) + Eqs. (PhiDefinition),
# (PsiDefinition): the continuation of a discrete plane wave into the layer
# is an exact eigenmode of one step, for ANY damping profile.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("k", [(0.7, 0.4), (2.5, 1.1), (0.3 + 0.2j, 0.9), (3.0, 0.05)])
def test_layer_mode_is_exact_one_step_eigenmode_2d(oracle_lib, k):
    oracle = oracle_lib
    rng = np.random.default_rng(11)
    N, b, h, dt = [26, 21], [12, 9], 1.0, 0.5
    sig = []
    for a in range(2):
        s = np.zeros(N[a])
        s[b[a]:] = rng.uniform(0.0, 2.0, size=N[a] - b[a])  # random profile (Fig. 3)
        sig.append(s)
    mode = cf.layer_mode(N, b, sig, k, h, dt)
    g = oracle.Grid(N, h, dt, sig)
    z = mode["z"]
    inner = (slice(1, -1), slice(1, -1))   # stencils that do not cross the array ends
    scale = max(np.max(np.abs(mode["U"])), 1.0)
    for part in (np.real, np.imag):
        s1 = oracle.step(g, _state_part(mode, part))
        assert np.max(np.abs(s1.U - part(z * mode["U"]))[inner]) <= 1e-13 * scale
        for a in range(2):
            assert np.max(np.abs(s1.Phi[a] - part(z * mode["Phi"][a]))[inner]) <= 1e-13 * scale
            assert np.max(np.abs(s1.Psi[a] - part(z * mode["Psi"][a]))[inner]) <= 1e-13 * scale


def test_layer_mode_is_exact_one_step_eigenmode_3d(oracle_lib):
    oracle = oracle_lib
    rng = np.random.default_rng(5)
    N, b, h, dt = [14, 12, 11], [6, 5, 4], 1.0, 0.4
    sig = []
    for a in range(3):
        s = np.zeros(N[a])
        s[b[a]:] = rng.uniform(0.0, 2.0, size=N[a] - b[a])
        sig.append(s)
    mode = cf.layer_mode(N, b, sig, (0.9, 0.5, 1.7), h, dt)
    g = oracle.Grid(N, h, dt, sig)
    z = mode["z"]
    inner = (slice(1, -1),) * 3
    for part in (np.real, np.imag):
        s1 = oracle.step(g, _state_part(mode, part))
        assert np.max(np.abs(s1.U - part(z * mode["U"]))[inner]) <= 1e-13
        for a in range(3):
            assert np.max(np.abs(s1.Phi[a] - part(z * mode["Phi"][a]))[inner]) <= 1e-13
            assert np.max(np.abs(s1.Psi[a] - part(z * mode["Psi"][a]))[inner]) <= 1e-13


def test_layer_mode_fails_for_wrong_time_frequency(oracle_lib):
    """The exactness above is sharp: building the mode with omega' = Omega
    (instead of i(z - 1)/dt) leaves an O(1e-2) defect, so the pin really
    constrains where the scheme evaluates its damping terms."""
    oracle = oracle_lib
    N, b, h, dt = [30], [10], 1.0, 0.5
    s = np.zeros(30)
    s[10:] = 1.0
    k = 0.8
    z = cf.step_factor([k], h, dt)
    omega = -np.angle(z) / dt
    good = cf.layer_mode(N, b, [s], [k], h, dt)
    U, Phi, Psi = cf._axis_factors(30, 10, s, k, omega, h)
    bad = {"U": U, "Uprev": U / z, "Phi": [Phi], "Psi": [Psi]}
    g = oracle.Grid(N, h, dt, [s])
    def defect(m):
        s1 = oracle.step(g, _state_part(m, np.real))
        return max(np.max(np.abs(s1.Phi[0] - np.real(z * m["Phi"][0]))[1:-1]),
                   np.max(np.abs(s1.Psi[0] - np.real(z * m["Psi"][0]))[1:-1]))
    # (the U equation alone holds for any omega' once Phi, Psi are built with
    # the same omega'; the auxiliary equations are what fix omega')
    assert defect(good) < 1e-14 and defect(bad) > 1e-4


# --------------------------------------------------------------------------
# Sec. 1.1.1 / Eq. (DiscreteDispersion): with sigma = 0 the scheme is the
# plain leapfrog wave equation; a periodic Fourier mode started at rest
# evolves as cos(n theta) exactly.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("ndim,dt", [(1, 0.9), (2, 0.5), (3, 0.4)])
def test_fourier_mode_exact(oracle_lib, ndim, dt):
    oracle = oracle_lib
    N = [24, 20, 16][:ndim]
    m = [3, 2, 5][:ndim]
    k = [2 * math.pi * m[a] / N[a] for a in range(ndim)]
    X = np.meshgrid(*[np.arange(n) for n in reversed(N)], indexing="ij")[::-1]
    U0 = np.cos(sum(k[a] * X[a] for a in range(ndim)))
    sig = [np.zeros(n) for n in N]
    g = oracle.Grid(N, 1.0, dt, sig)
    theta = cf.leapfrog_theta(k, 1.0, dt)
    s = oracle.start(g, U0)
    assert np.max(np.abs(s.Uprev - math.cos(theta) * U0)) < 1e-14
    steps = 300
    fin, _ = oracle.run(g, s, steps)
    assert np.max(np.abs(fin.U - math.cos(steps * theta) * U0)) < 5e-13
    # ... and for the plain wave reference run
    Uw, _ = oracle.wave_run(g, s.U, s.Uprev, steps)
    assert np.max(np.abs(Uw - math.cos(steps * theta) * U0)) < 5e-13


@pytest.mark.parametrize("ndim,dt,amp,vel", [(1, 0.9, 1.0, 0.7), (1, 0.6, 0.0, 1.0),
                                             (2, 0.5, 0.8, -1.3), (2, 0.5, 0.0, 0.5),
                                             (3, 0.4, 1.0, 0.9), (3, 0.4, 0.0, -2.0)])
def test_fourier_mode_with_initial_velocity_exact(oracle_lib, ndim, dt, amp, vel):
    """The start with a given velocity.  With sigma = 0 the leapfrog
    recurrence U^{n+1} = (2 - 4 sin^2(theta/2)) U^n - U^{n-1} on a periodic
    Fourier mode (Sec. 1.1.1, Eq. DiscreteDispersion: sin(theta/2) =
    (c dt/h) sqrt(sum sin^2(k h/2))) has the general solution
    A cos(n theta) + B sin(n theta).  U^0 = a cos(k.x) gives A = a; a start
    U^{-1} = U^0 - dt V^0 + dt^2/2 A(U^0) with V^0 = v cos(k.x) gives
    U^{-1} = a cos(theta) - dt v, hence B = dt v / sin(theta).  A flipped sign
    or a dropped dt on the velocity term changes B and fails this."""
    oracle = oracle_lib
    N = [24, 20, 16][:ndim]
    m = [3, 2, 5][:ndim]
    k = [2 * math.pi * m[a] / N[a] for a in range(ndim)]
    X = np.meshgrid(*[np.arange(n) for n in reversed(N)], indexing="ij")[::-1]
    mode = np.cos(sum(k[a] * X[a] for a in range(ndim)))
    g = oracle.Grid(N, 1.0, dt, [np.zeros(n) for n in N])
    theta = cf.leapfrog_theta(k, 1.0, dt)
    B = dt * vel / math.sin(theta)
    s = oracle.start(g, amp * mode, vel * mode)
    # level -1 of the closed form: a cos(theta) - B sin(theta)
    assert np.max(np.abs(s.Uprev - (amp * math.cos(theta) - B * math.sin(theta)) * mode)) < 1e-14
    steps = 300
    fin, _ = oracle.run(g, s, steps)
    want = (amp * math.cos(steps * theta) + B * math.sin(steps * theta)) * mode
    assert np.max(np.abs(fin.U - want)) < 5e-13
    want_prev = (amp * math.cos((steps - 1) * theta) + B * math.sin((steps - 1) * theta)) * mode
    assert np.max(np.abs(fin.Uprev - want_prev)) < 5e-13


def test_fourier_mode_exact_with_constant_c2(oracle_lib):
    """c^2 multiplies the Laplacian: a constant c0^2 rescales the phase
    advance to sin(theta/2) = (c0 dt/h) sqrt(sum sin^2(k h/2))."""
    oracle = oracle_lib
    N = [32, 24]
    k = [2 * math.pi * 5 / 32, 2 * math.pi * 2 / 24]
    X = np.meshgrid(np.arange(24), np.arange(32), indexing="ij")[::-1]
    U0 = np.cos(k[0] * X[0] + k[1] * X[1])
    c0 = 0.8
    g = oracle.Grid(N, 1.0, 0.5, [np.zeros(32), np.zeros(24)], c2=np.full((24, 32), c0 * c0))
    theta = cf.leapfrog_theta(k, 1.0, 0.5, c=c0)
    fin, _ = oracle.run(g, oracle.start(g, U0), 200)
    assert np.max(np.abs(fin.U - math.cos(200 * theta) * U0)) < 5e-13


# --------------------------------------------------------------------------
# Eq. (Energy): without damping on a periodic grid the (time-staggered)
# spring-mass energy is conserved by leapfrog, also with a variable c^2.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("variable_c2", [False, True])
def test_energy_conserved_without_damping(oracle_lib, variable_c2):
    oracle = oracle_lib
    rng = np.random.default_rng(3)
    n, N = [40, 36], [40, 36]
    U0 = synthetic.gaussian_sum(n, [0, 0], [0, 0], 12, 2.0, 5.0, rng)
    c2 = None
    if variable_c2:
        c2 = synthetic.smooth_c2(n, [0, 0], [0, 0], 6, 4.0, 9.0, 0.5, 0, rng)
    g = oracle.Grid(N, 1.0, 0.45, [np.zeros(40), np.zeros(36)], c2=c2)
    s = oracle.start(g, U0)
    energies = []
    for _ in range(5):
        s2, _ = oracle.run(g, s, 100)
        one, _ = oracle.run(g, s2, 1)
        energies.append(cf.leapfrog_energy(one.U, s2.U, 1.0, 0.45, c2=c2))
        s = s2
    e = np.array(energies)
    assert np.max(np.abs(e - e[0])) / e[0] < 1e-13


# --------------------------------------------------------------------------
# Figs. 2 and 3: reflection measured as max|U - U_ref| in the physical domain
# against the untruncated free-space run, before any wave can cross the layer
# and come back (so the difference is pure interface reflection).
# --------------------------------------------------------------------------
def _reflection(oracle, n, m, steps, sigma, make_u0, norm="final"):
    """max|U - U_ref| over the physical domain after ``steps`` steps, divided by
    the reference peak at that step (``norm="final"``) or by the initial peak
    (``norm="initial"``, the paper's absolute measure for a fixed bump)."""
    N = n + 2 * m
    g = oracle.Grid([N, N], 1.0, 0.5, [sigma, sigma.copy()])
    fin, _ = oracle.run(g, oracle.start(g, make_u0([n, n], [m, m], [m, m])), steps)
    Nr = n + 2 * (steps + 4)
    off = (Nr - n) // 2
    gr = oracle.Grid([Nr, Nr], 1.0, 0.5, [None, None])
    sr = oracle.start(gr, make_u0([n, n], [off, off], [Nr - n - off] * 2))
    Ur, _ = oracle.wave_run(gr, sr.U, sr.Uprev, steps)
    a = fin.U[m:m + n, m:m + n]
    r = Ur[off:off + n, off:off + n]
    peak = np.max(np.abs(r)) if norm == "final" else np.max(np.abs(sr.U))
    return np.max(np.abs(a - r)) / peak


def _paper_setups():
    with open(os.path.join(GOLDEN, "paper_setups.json")) as f:
        return json.load(f)


def test_reflectionless_fig2_constant_damping(oracle_lib):
    cfg = _paper_setups()["fig2"]
    n, m, steps = cfg["interior_cells"], cfg["layer_cells_per_side"], cfg["steps"]
    sig = synthetic.sigma_const(n, m, m, cfg["sigma_h"])
    err = _reflection(oracle_lib, n, m, steps, sig,
                      lambda nn, lo, hi: synthetic.gaussian_bump(nn, lo, hi, cfg["bump_width"],
                                                                 amp=cfg["bump_peak"]))
    assert err < 1e-13


def test_reflectionless_fig3_random_damping_white_noise(oracle_lib):
    cfg = _paper_setups()["fig3"]
    n, m, steps = cfg["interior_cells"], cfg["layer_cells_per_side"], cfg["steps"]
    sig = synthetic.sigma_random(n, m, m, cfg["sigma_h_max"], np.random.default_rng(cfg["seed"]))
    err = _reflection(oracle_lib, n, m, steps, sig,
                      lambda nn, lo, hi: synthetic.white_noise_disk(
                          nn, lo, hi, n * cfg["disk_radius_fraction"], cfg["variance"],
                          np.random.default_rng(cfg["seed"] + 1)))
    assert err < 1e-13


def test_reflection_detects_a_wrong_layer(oracle_lib):
    """Control for the two tests above: a damping profile that is NOT the
    paper's layer (sigma applied to the auxiliaries only through one of the two
    coupling terms) is visibly reflecting under the same measurement."""
    oracle = oracle_lib
    n, m, steps = 80, 40, 80
    sig = synthetic.sigma_const(n, m, m, 2.0)
    # naive absorbing layer: plain wave equation plus a local damping of U
    N = n + 2 * m
    g0 = oracle.Grid([N, N], 1.0, 0.5, [None, None])
    s = oracle.start(g0, synthetic.gaussian_bump([n, n], [m, m], [m, m], 4.0))
    damp = np.add.outer(sig, sig)
    U, Up = s.U, s.Uprev
    for _ in range(steps):
        Un, _ = oracle.wave_run(g0, U, Up, 1)
        Un = U + (Un - U) / (1.0 + 0.5 * 0.5 * damp)
        U, Up = Un, U
    Nr = n + 2 * (steps + 4)
    off = (Nr - n) // 2
    gr = oracle.Grid([Nr, Nr], 1.0, 0.5, [None, None])
    sr = oracle.start(gr, synthetic.gaussian_bump([n, n], [off, off], [Nr - n - off] * 2, 4.0))
    Ur, _ = oracle.wave_run(gr, sr.U, sr.Uprev, steps)
    err = np.max(np.abs(U[m:m + n, m:m + n] - Ur[off:off + n, off:off + n])) / np.max(np.abs(Ur))
    assert err > 1e-4


# --------------------------------------------------------------------------
# Fig. 5(c): the residual (round-trip) wave falls exponentially as the layer
# thickens linearly (sigma = 1/h).
# --------------------------------------------------------------------------
def test_residual_decays_exponentially_with_thickness(oracle_lib):
    cfg = _paper_setups()["fig5c"]
    errs = []
    n = cfg["interior_cells"]
    for m in cfg["thicknesses"]:
        sig = synthetic.sigma_const(n, m, m, cfg["sigma_h"])
        errs.append(_reflection(oracle_lib, n, m, cfg["steps"], sig,
                                lambda nn, lo, hi: synthetic.gaussian_bump(nn, lo, hi, cfg["bump_width"]),
                                norm="initial"))
    errs = np.array(errs)
    # falls by more than 1e2 per 4 extra cells until it reaches rounding level
    for a, b in zip(errs[:-1], errs[1:]):
        assert b < 1e-2 * a or b < 1e-15
    assert errs[-1] < 1e-15


# --------------------------------------------------------------------------
# Fig. 6: long runs stay bounded; the energy left in the physical domain decays.
# --------------------------------------------------------------------------
@pytest.mark.parametrize("profile", ["const", "random"])
def test_long_run_bounded_energy_decays(oracle_lib, profile):
    oracle = oracle_lib
    cfg = _paper_setups()["fig6"]
    n, m = cfg["interior_cells"], cfg["layer_cells_per_side"]
    if profile == "const":
        sig = [synthetic.sigma_const(n, m, m, cfg["sigma_h"])] * 2
    else:
        rng = np.random.default_rng(cfg["seed"])
        sig = [synthetic.sigma_random(n, m, m, cfg["sigma_h"], rng) for _ in range(2)]
    N = n + 2 * m
    g = oracle.Grid([N, N], 1.0, 0.5, sig)
    s = oracle.start(g, synthetic.gaussian_bump([n, n], [m, m], [m, m], cfg["bump_width"]))
    box = (slice(m, m + n), slice(m, m + n))
    e0 = cf.leapfrog_energy(s.U, s.Uprev, 1.0, 0.5, box=box)
    peak = [np.max(np.abs(s.U))]
    for _ in range(cfg["chunks"]):
        s2, _ = oracle.run(g, s, cfg["chunk_steps"] - 1)
        s3, _ = oracle.run(g, s2, 1)
        e = cf.leapfrog_energy(s3.U, s2.U, 1.0, 0.5, box=box)
        peak.append(np.max(np.abs(s3.U)))
        s = s3
    assert np.all(np.isfinite(peak))
    assert e < 1e-9 * e0
    assert max(peak[1:]) <= peak[0]


# --------------------------------------------------------------------------
# Point sources: 1-D leapfrog at Courant number 1 is an exact shift, so an
# impulse injected in the first step spreads as the discrete light cone.
# --------------------------------------------------------------------------
def test_point_source_light_cone_1d(oracle_lib):
    oracle = oracle_lib
    N, src, steps = 101, 50, 40
    g = oracle.Grid([N], 1.0, 1.0, [np.zeros(N)])
    s = oracle.start(g, np.zeros(N))
    wav = np.zeros((1, steps))
    wav[0, 0] = 1.0                       # dt^2 w / h = 1: U^1 = delta at src
    rec = [40, 47, 50, 53, 60, 75]
    fin, tr = oracle.run(g, s, steps, sources=[src], wavelets=wav, receivers=rec, nt=steps)
    expected_final = cf.green_1d_cfl1(steps, np.arange(N) - src)
    assert np.array_equal(fin.U, expected_final)
    for r, cell in enumerate(rec):
        for n in range(steps):
            assert tr[r, n] == cf.green_1d_cfl1(n + 1, np.array([cell - src]))[0]


# --------------------------------------------------------------------------
# Sec. 1.1.2: Phi_a is only needed on the layer {i_a >= 0} and Psi_a on
# {i_a >= 1}; zeroing them elsewhere after every step changes nothing
# (the GPU stores them only there).
# --------------------------------------------------------------------------
def test_auxiliaries_outside_their_support_are_inert(oracle_lib):
    oracle = oracle_lib
    n, lo, hi = 24, 6, 5
    N = lo + n + hi
    rng = np.random.default_rng(2)
    sig = [synthetic.sigma_random(n, lo, hi, 2.0, rng) for _ in range(2)]
    g = oracle.Grid([N, N], 1.0, 0.5, sig)
    s = oracle.start(g, synthetic.gaussian_bump([n, n], [lo, lo], [hi, hi], 3.0))
    ref, _ = oracle.run(g, s, 60)
    band = np.array([((i - (lo + n)) % N) for i in range(N)])
    phi_sup = band <= lo + hi - 1
    psi_sup = (band >= 1) & (band <= lo + hi)
    t = s
    for _ in range(60):
        t = oracle.step(g, t)
        t.Phi[0][:, ~phi_sup] = 0.0
        t.Phi[1][~phi_sup, :] = 0.0
        t.Psi[0][:, ~psi_sup] = 0.0
        t.Psi[1][~psi_sup, :] = 0.0
    assert np.max(np.abs(t.U - ref.U)) < 1e-15
    assert np.max(np.abs(t.Phi[0][:, phi_sup] - ref.Phi[0][:, phi_sup])) < 1e-15
    assert np.max(np.abs(t.Psi[1][psi_sup, :] - ref.Psi[1][psi_sup, :])) < 1e-15


# --------------------------------------------------------------------------
# Thm. 1: the result does not depend on the orientation of the equations:
# a mirror-symmetric bump stays mirror symmetric in the physical domain.
# --------------------------------------------------------------------------
def test_mirror_symmetry_of_interior_field(oracle_lib):
    oracle = oracle_lib
    n, m, steps = 60, 40, 70
    sig = synthetic.sigma_const(n, m, m, 2.0)
    N = n + 2 * m
    g = oracle.Grid([N, N], 1.0, 0.5, [sig, sig.copy()])
    fin, _ = oracle.run(g, oracle.start(g, synthetic.gaussian_bump([n, n], [m, m], [m, m], 3.0)), steps)
    a = fin.U[m:m + n, m:m + n]
    pk = np.max(np.abs(a))
    assert np.max(np.abs(a - a[:, ::-1])) < 1e-13 * pk
    assert np.max(np.abs(a - a[::-1, :])) < 1e-13 * pk
    assert np.max(np.abs(a - a.T)) < 1e-13 * pk


# --------------------------------------------------------------------------
# Thm. 3 (Eqs. IntroDecayBound, IntroReflectedDecayBound) and the special
# cases of App. A: properties of the closed form the pins above rely on.
# --------------------------------------------------------------------------
def test_rho_bounds_and_special_cases():
    h = 1.0
    rng = np.random.default_rng(0)
    s = rng.uniform(1e-3, 4.0, size=2000)
    w = rng.uniform(1e-2, 3.0, size=2000)
    kr = rng.uniform(1e-3, math.pi - 1e-3, size=2000)
    ki = -rng.uniform(0.0, 2.0, size=2000)
    k = kr + 1j * ki
    r = cf.rho(s, k, w, h)
    assert np.all(np.abs(r) < 1.0)
    assert np.all(np.abs(r) / np.abs(cf.rho(s, -np.conj(k), w, h)) < 1.0)
    # negative frequency: sgn(omega) Re(k) in (0, pi) means Re(k) < 0
    assert np.all(np.abs(cf.rho(s, -kr, -w, h)) < 1.0)
    assert np.allclose(cf.rho(0.0, k, w, h), 1.0, atol=0, rtol=1e-15)   # zero gap (Lemma)
    assert np.allclose(cf.rho(s, 0.0, w, h), 1.0, atol=1e-15)           # case k = 0
    assert np.allclose(cf.rho(s, math.pi / h, w, h), 1.0, atol=1e-14)   # case k = pi/h
    # smooth asymptotics, Eq. (RhoAsymptotics): the (1,1)-Pade of
    # exp(-sigma h k/omega) is the limit, with an O(kh) correction
    errs = []
    for kk in (1e-2, 1e-3, 1e-4):
        ww = 2.0 * math.sin(kk / 2.0)        # 1-D dispersion, h = 1
        pade = (2.0 - 1.0 * kk / ww) / (2.0 + 1.0 * kk / ww)
        errs.append(abs(cf.rho(1.0, kk, ww) - pade))
    assert errs[0] < 0.2 * 1e-2 and 5.0 < errs[0] / errs[1] < 20.0 and 5.0 < errs[1] / errs[2] < 20.0


def test_golden_oracle_regression(oracle_lib):
    """Sampled values of the 128^2 + 16-cell bump run, written by
    tests/golden/make_golden.py (which calls only the oracle)."""
    oracle = oracle_lib
    with open(os.path.join(GOLDEN, "bump2d_128_m16_samples.json")) as f:
        gold = json.load(f)
    w = synthetic.bump2d(128, 16, gold["steps"])
    g = oracle.Grid(w.N, w.h, w.dt, w.sigma)
    fin, _ = oracle.run(g, oracle.start(g, w.U0), gold["steps"])
    for (y, x), v in zip(gold["cells"], gold["U"]):
        assert abs(fin.U[y, x] - v) <= 1e-14 * max(1.0, abs(v))
