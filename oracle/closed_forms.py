"""Closed forms from the paper, used to pin the oracle (test infrastructure).

Nothing here time-steps anything; these are the paper's explicit formulas,
evaluated in complex FP64:

* ``rho``              -- the one-cell decay factor, Eq. (IntroDecayRate) /
                          Eq. (DecayRate) of Thm. 2.
* ``leapfrog_theta``   -- phase advance per step of a periodic Fourier mode of
                          the leapfrog discretisation of Eq. (DiscreteWaveEquation)
                          (spatial symbol from Eq. (DiscreteDispersion)).
* ``layer_mode``       -- the unique continuation of a discrete plane wave
                          into the layer (Thm. 1, Eq. (IntroSolution)), with the
                          auxiliaries built from their definitions as scaled
                          discrete complex derivatives on the parallelogram
                          graph, Eqs. (PhiDefinition), (PsiDefinition).
* ``green_1d_cfl1``    -- the 1-D leapfrog Green's function at Courant number 1
                          (the scheme is then an exact shift: d'Alembert).
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np


def rho(s, k, omega, h=1.0):
    """rho(s, k, omega) = (2 + i s/omega (1 - e^{-ikh})) / (2 + i s/omega (1 - e^{ikh})),
    Eq. (IntroDecayRate).  Accepts complex omega (the time-discrete frequency)."""
    s = np.asarray(s, dtype=np.complex128)
    k = np.asarray(k, dtype=np.complex128)
    omega = np.asarray(omega, dtype=np.complex128)
    num = 2.0 + 1j * (s / omega) * (1.0 - np.exp(-1j * k * h))
    den = 2.0 + 1j * (s / omega) * (1.0 - np.exp(1j * k * h))
    return num / den


def leapfrog_theta(k: Sequence[float], h: float, dt: float, c: float = 1.0) -> float:
    """Phase advance theta per step of cos(k.x) under the leapfrog scheme:
    sin(theta/2) = (c dt/h) sqrt(sum_a sin^2(k_a h/2))."""
    s = math.sqrt(sum(math.sin(ka * h / 2.0) ** 2 for ka in k))
    return 2.0 * math.asin(c * dt / h * s)


def step_factor(k: Sequence[complex], h: float, dt: float) -> complex:
    """One-step amplification z = e^{-i Omega dt} of the time-discrete plane
    wave with wave numbers k (unit speed): z solves
    (z - 2 + 1/z)/dt^2 = -sum_a (4/h^2) sin^2(k_a h/2)."""
    lam = sum((4.0 / h ** 2) * np.sin(np.complex128(ka) * h / 2.0) ** 2 for ka in k)
    b = 2.0 - dt * dt * lam            # z + 1/z = b
    disc = np.sqrt(np.complex128(b * b - 4.0))
    z1 = (b - disc) / 2.0
    z2 = (b + disc) / 2.0
    # pick the root with negative phase (e^{-i Omega dt}, Omega > 0)
    return z1 if np.angle(z1) < 0 else z2


def _axis_factors(N: int, b: int, sig: np.ndarray, k: complex, wp: complex, h: float):
    """Per-axis factors of the layer mode along one axis with extent N whose
    paper origin (first layer cell, p = 0) sits at array index b.
    Returns (U_a, Phi_a, Psi_a) as complex arrays of length N."""
    i = np.arange(N)
    p = i - b
    W = lambda q: np.exp(1j * k * h * q)            # W_k(q) = e^{ikhq}
    r = rho(sig, k, wp, h)                          # rho at each array index
    # R(p) = prod_{j=0}^{p-1} rho(sigma(j)) for p > 0, 1 for p <= 0
    R = np.ones(N, dtype=np.complex128)
    for idx in range(N):
        if p[idx] > 0:
            R[idx] = R[idx - 1] * r[idx - 1]
    Rm1 = np.ones(N, dtype=np.complex128)           # R(p - 1)
    Rm1[1:] = R[:-1]
    sig_left = np.zeros(N)                          # sigma(p - 1)
    sig_left[1:] = sig[:-1]
    U = R * W(p)
    # Eq. (PhiDefinition B): Phi_hat(p) = -(f(-1,p+1) - f(0,p)) / (sigma(p) h)
    #   = W(p) R(p) (1 - rho_p)/(sigma_p h) = W(p) R(p) 2 sin(kh) / (omega' h D_p)
    D = 2.0 + 1j * (sig / wp) * (1.0 - np.exp(1j * k * h))
    Phi = W(p) * R * 2.0 * np.sin(k * h) / (wp * h * D)
    # Eq. (PsiDefinition A): Psi_hat(p) = (f(1,p) - f(0,p-1)) / (i omega' h (2 + i sigma(p-1)/omega'))
    Psi = (R * W(p + 1) - Rm1 * W(p - 1)) / (1j * wp * h * (2.0 + 1j * sig_left / wp))
    return U, Phi, Psi


def layer_mode(N: Sequence[int], b: Sequence[int], sigma: Sequence[np.ndarray],
               k: Sequence[complex], h: float, dt: float):
    """Exact time-harmonic solution of the fully discrete scheme (leapfrog for
    U, forward step for the auxiliaries, all right-hand sides at time n):
    the discrete plane wave prod_a W_{k_a} continued into the layer by
    Thm. 1, with omega' = i (z - 1)/dt.

    ``N``, ``b``, ``sigma``, ``k`` are per axis in the paper's order (x, y, z);
    sigma[a] must vanish at array indices < b[a].  Returns a dict with complex
    arrays of numpy shape (reversed N): U (time n), Uprev (time n-1), Phi,
    Psi (lists per axis, time n) and the step factor z, so that one step maps
    (U, Uprev, Phi, Psi) to (z U, U, z Phi, z Psi) away from the array ends.
    """
    d = len(N)
    z = step_factor(k, h, dt)
    wp = 1j * (z - 1.0) / dt
    facs = [_axis_factors(int(N[a]), int(b[a]), np.asarray(sigma[a], dtype=np.float64),
                          np.complex128(k[a]), wp, h) for a in range(d)]

    def outer(parts):
        # parts[a] is the factor along axis a; numpy axis order is reversed
        out = np.ones((), dtype=np.complex128)
        for a in reversed(range(d)):
            out = np.multiply.outer(out, parts[a])
        return out

    U = outer([f[0] for f in facs])
    Phi, Psi = [], []
    for a in range(d):
        Phi.append(outer([facs[c][1] if c == a else facs[c][0] for c in range(d)]))
        Psi.append(outer([facs[c][2] if c == a else facs[c][0] for c in range(d)]))
    return {"U": U, "Uprev": U / z, "Phi": Phi, "Psi": Psi, "z": z, "omega_prime": wp}


def green_1d_cfl1(n: int, i: np.ndarray) -> np.ndarray:
    """1-D leapfrog at Courant number 1 with U^0 = 0, U^1 = delta_0 (an impulse
    injected in the first step): U^n(i) = 1 where |i| <= n-1 and i = n-1 (mod 2),
    else 0 (the discrete d'Alembert light cone)."""
    i = np.asarray(i)
    return ((np.abs(i) <= n - 1) & ((i - (n - 1)) % 2 == 0)).astype(np.float64)


def leapfrog_energy(U_new: np.ndarray, U_old: np.ndarray, h: float, dt: float,
                    c2=None, box=None, walls=False) -> float:
    """Spring-mass energy of Eq. (Energy) in the time-staggered form that the
    leapfrog scheme conserves (periodic grid, no damping):
    E^{n+1/2} = 1/2 sum |(U^{n+1} - U^n)/dt|^2 / c^2
              + 1/2 sum_a <D_a U^{n+1}, D_a U^n> / h^2,   D_a U = tau_a U - U.
    ``box`` (tuple of numpy slices) restricts the sums to a sub-box (the
    physical domain) -- then it is a diagnostic, not a conserved quantity."""
    v = (U_new - U_old) / dt
    kin = v * v if c2 is None else v * v / c2
    if walls:
        # Dirichlet ghosts at -1 and N on every axis: sum over all edges,
        # including the two boundary edges of each line
        if box is not None:
            raise ValueError("box and walls are exclusive")
        pot = 0.0
        for ax in range(U_new.ndim):
            pad = [(0, 0)] * U_new.ndim
            pad[ax] = (1, 1)
            dn = np.diff(np.pad(U_new, pad), axis=ax)
            do = np.diff(np.pad(U_old, pad), axis=ax)
            pot += float(np.sum(dn * do)) / (h * h)
        return 0.5 * float(np.sum(kin)) + 0.5 * pot
    pot = np.zeros_like(U_new)
    for ax in range(U_new.ndim):
        dn = np.roll(U_new, -1, axis=ax) - U_new
        do = np.roll(U_old, -1, axis=ax) - U_old
        pot += dn * do / (h * h)
    if box is not None:
        kin = kin[box]
        pot = pot[box]
    return 0.5 * float(np.sum(kin)) + 0.5 * float(np.sum(pot))


def semidiscrete_layer_mode(N, b, sigma, k, h: float):
    """Exact solution of the semi-discrete system (continuous time) of
    Eq. (DiscretePML): the plane wave prod_a W_{k_a} e^{-i omega t} with
    omega^2 h^2 = sum_a 4 sin^2(k_a h/2) (Eq. DiscreteDispersion), continued
    into the layer by Thm. 1 (omega' = omega).  Returns U, V = -i omega U, Phi,
    Psi at t = 0 and omega; any one-step method that is a polynomial P in the
    system matrix (RK4: P(x) = 1 + x + x^2/2 + x^3/6 + x^4/24) maps it to
    P(-i omega dt) times itself."""
    d = len(N)
    lam = sum((4.0 / h ** 2) * np.sin(np.complex128(ka) * h / 2.0) ** 2 for ka in k)
    omega = np.sqrt(np.complex128(lam))
    facs = [_axis_factors(int(N[a]), int(b[a]), np.asarray(sigma[a], dtype=np.float64),
                          np.complex128(k[a]), omega, h) for a in range(d)]

    def outer(parts):
        out = np.ones((), dtype=np.complex128)
        for a in reversed(range(d)):
            out = np.multiply.outer(out, parts[a])
        return out

    U = outer([f[0] for f in facs])
    Phi = [outer([facs[c][1] if c == a else facs[c][0] for c in range(d)]) for a in range(d)]
    Psi = [outer([facs[c][2] if c == a else facs[c][0] for c in range(d)]) for a in range(d)]
    return {"U": U, "V": -1j * omega * U, "Phi": Phi, "Psi": Psi, "omega": omega}


def rk4_factor(x: complex) -> complex:
    """Amplification polynomial of classic RK4 for y' = lambda y, x = lambda dt."""
    return 1.0 + x + x * x / 2.0 + x ** 3 / 6.0 + x ** 4 / 24.0
