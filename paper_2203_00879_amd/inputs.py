"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module holds no derivative, right-hand-side or time-stepping arithmetic:
it builds initial states and test fields only, with numpy, from a seed.

* ``AIR``: SI parameters of the Rayleigh-Taylor box (Section 2: air, gamma =
  1.4, Pr = 0.712, box edge L = 0.15 m, T_s = 300 K; Sutherland constants and
  the bulk-viscosity regression, eq. reg).  rho_s = p_int / (R T_s) so that the
  interface pressure 101325 Pa is the non-dimensional reference pressure.
* ``rti_state``: two resting air masses at different temperatures separated
  at mid-height, hydrostatic in each half with equal pressure at the interface
  (Section 2 and Fig. 1), the two interface planes' temperature perturbed by
  seeded uniform noise.
* ``fourier_field``: a sum of seeded random 3D Fourier modes with analytic
  first and second derivatives.

Non-dimensional state layout (the library's and the oracle's): float64 array
``Q[5, nz, ny, nx]`` = [rho, rho u, rho v, rho w, E'] with
``E' = rho e_t - Rh/(gamma-1)``, ``Rh = R T_s / (g L)``; x fastest, y up.
"""
import math

import numpy as np

P_INT = 101325.0

AIR = dict(
    gamma=1.4, R_gas=287.0, g=9.81, L=0.15, T_s=300.0, rho_s=P_INT / (287.0 * 300.0), Pr=0.712,
    mu_ref=1.716e-5, T_ref=273.15, S_suth=110.4, mub_a=3.381e-4, mub_b=7.383e-4, viscous=1, gravity=1,
)


def rh_of(params):
    """Non-dimensional gas constant R T_s / (g L) (the reference pressure p_int)."""
    return params["R_gas"] * params["T_s"] / (params["g"] * params["L"])


def rti_state(n, T_upper=300.0, T_lower=500.0, params=AIR, seed=0, noise_K=1e-6, length=1.0):
    """Rayleigh-Taylor initial state on an (nx, ny, nz) = n box with nodes on the walls.

    Upper half (j >= ny // 2) at T_upper, lower half at T_lower (kelvin), at rest;
    p = p_int exp(-(y - len_y/2) / (Rh T_half)) in each half (non-dimensional,
    g L / U_s^2 = 1); the planes j = ny//2 - 1 and ny//2 get T += noise_K * U(-1, 1)
    drawn from ``numpy.random.default_rng(seed)`` with shape (2, nz, nx).
    Returns Q[5, nz, ny, nx].
    """
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    lx, ly, lz = (length,) * 3 if np.isscalar(length) else length
    gamma = params["gamma"]
    Rh = rh_of(params)
    Ts = params["T_s"]
    y = np.arange(ny, dtype=np.float64) * (ly / (ny - 1))
    upper = np.arange(ny) >= ny // 2
    Th = np.where(upper, T_upper / Ts, T_lower / Ts)
    arg = -(y - 0.5 * ly) / (Rh * Th)
    T = np.broadcast_to(Th[None, :, None], (nz, ny, nx)).copy()
    if noise_K:
        rng = np.random.default_rng(seed)
        noise = rng.uniform(-1.0, 1.0, size=(2, nz, nx)) * (noise_K / Ts)
        T[:, ny // 2 - 1, :] += noise[0]
        T[:, ny // 2, :] += noise[1]
    Q = np.zeros((5, nz, ny, nx), dtype=np.float64)
    Q[0] = np.exp(arg)[None, :, None] / T                      # rho = p / (Rh T)
    Q[4] = np.broadcast_to((Rh * np.expm1(arg) / (gamma - 1.0))[None, :, None], (nz, ny, nx))
    return Q


def uniform_state(n, T=1.0, rho=1.0, velocity=(0.0, 0.0, 0.0), params=AIR):
    """Uniform state (non-dimensional T and rho)."""
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    gamma = params["gamma"]
    Rh = rh_of(params)
    Q = np.zeros((5, nz, ny, nx))
    Q[0] = rho
    for d in range(3):
        Q[1 + d] = rho * velocity[d]
    ke = 0.5 * rho * sum(v * v for v in velocity)
    Q[4] = (Rh * (rho * T - 1.0)) / (gamma - 1.0) + ke
    return Q


def fourier_modes(nmodes=16, kmax=64, seed=1):
    """Mode list [(kx, ky, kz, a, phi)], drawn per mode in that order from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    modes = []
    for _ in range(nmodes):
        kx = int(rng.integers(1, kmax + 1))
        ky = int(rng.integers(1, kmax + 1))
        kz = int(rng.integers(1, kmax + 1))
        a = float(rng.normal())
        phi = float(rng.uniform(0.0, 2.0 * math.pi))
        modes.append((kx, ky, kz, a, phi))
    return modes


def fourier_field(n, modes, which=None, length=1.0, dtype=np.float64, factor=None):
    """f = sum_m a_m cos(2 pi (kx x + ky y + kz z) + phi_m) on nodes x_i = i len/(n-1).

    which: None for f; (d, 1) or (d, 2) for the analytic first or second
    derivative along d (0 = x, 1 = y, 2 = z).  factor: optional function of the
    angular wavenumber w = 2 pi k_d that replaces w in the derivative (a Fourier
    multiplier).  Returns an array [nz, ny, nx].
    """
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    lx, ly, lz = (length,) * 3 if np.isscalar(length) else length
    x = np.arange(nx) * (lx / (nx - 1))
    y = np.arange(ny) * (ly / (ny - 1))
    z = np.arange(nz) * (lz / (nz - 1))
    out = np.zeros((nz, ny, nx), dtype=np.float64)
    for kx, ky, kz, a, phi in modes:
        k = (kx, ky, kz)
        # separable evaluation: cos(A + B + C) via complex exponentials
        ex = np.exp(1j * 2.0 * math.pi * kx * x)
        ey = np.exp(1j * 2.0 * math.pi * ky * y)
        ez = np.exp(1j * (2.0 * math.pi * kz * z + phi))
        e = ez[:, None, None] * ey[None, :, None] * ex[None, None, :]
        if which is None:
            out += a * e.real
        else:
            d, order = which
            w = 2.0 * math.pi * k[d]
            if factor is not None:
                w = factor(w)
            if order == 1:
                out += -a * w * e.imag
            else:
                out += -a * w * w * e.real
    return out.astype(dtype, copy=False)


def stable_dt(n, T_max_K, params=AIR, length=1.0):
    """Fixed time step from the initial state: 0.5 min(acoustic, viscous) bound.

    Acoustic: 2 sqrt(2) h / (k* sum_d c) with k* = 2.2090 the largest modified
    wavenumber of the interior scheme times h and c = sqrt(T/T_s)/M at the
    hottest temperature; viscous: 2.785 h^2 / (3 nu) with nu the largest
    (4/3 mu + mu_b/mu_s)/(rho Re).  A heuristic step-size rule, not part of the
    method.
    """
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    L = length
    h = min(L / (nx - 1), L / (ny - 1), L / (nz - 1))
    g, Lm, R, Ts, gam = params["g"], params["L"], params["R_gas"], params["T_s"], params["gamma"]
    Us = math.sqrt(g * Lm)
    M = Us / math.sqrt(gam * R * Ts)
    T = T_max_K / Ts
    c = math.sqrt(T) / M
    dt_ac = 2.0 * math.sqrt(2.0) * h / (2.2090 * 3.0 * c)
    r = T_max_K / params["T_ref"]
    mu_dim = params["mu_ref"] * r * math.sqrt(r) * (params["T_ref"] + params["S_suth"]) / (T_max_K + params["S_suth"])
    r_s = Ts / params["T_ref"]
    mu_s = params["mu_ref"] * r_s * math.sqrt(r_s) * (params["T_ref"] + params["S_suth"]) / (Ts + params["S_suth"])
    Re = params["rho_s"] * Us * Lm / mu_s
    beta = max(0.0, (params["mub_a"] * T_max_K - params["mub_b"]) / mu_s)
    rho_min = Ts / T_max_K * 0.9
    nu = ((4.0 / 3.0) * mu_dim / mu_s + beta) / (rho_min * Re)
    dt_v = 2.785 * h * h / (3.0 * nu) if params.get("viscous", 1) else float("inf")
    return 0.5 * min(dt_ac, dt_v)


def smooth_state(n, seed=0, amp_rho=0.2, amp_u=0.05, amp_p=0.5, kmax=3, params=AIR, length=1.0):
    """Smooth random state from (rho, u, v, w, p') built of a few low Fourier modes.

    rho = 1 + amp_rho s0, velocities amp_u s1..s3, p' = amp_p s4 with s_m smooth
    fields of unit scale; E' = p'/(gamma - 1) + rho |V|^2 / 2.  Returns Q[5, nz, ny, nx].
    """
    nx, ny, nz = (n, n, n) if np.isscalar(n) else n
    lx, ly, lz = (length,) * 3 if np.isscalar(length) else length
    rng = np.random.default_rng(seed)
    x = np.arange(nx) * (lx / (nx - 1))
    y = np.arange(ny) * (ly / (ny - 1))
    z = np.arange(nz) * (lz / (nz - 1))

    def field():
        out = np.zeros((nz, ny, nx))
        for _ in range(3):
            k = rng.integers(0, kmax + 1, size=3)
            ph = rng.uniform(0, 2 * math.pi, size=3)
            a = rng.uniform(-1, 1) / 3.0
            out += a * (np.cos(2 * math.pi * k[2] * z + ph[2])[:, None, None]
                        * np.cos(2 * math.pi * k[1] * y + ph[1])[None, :, None]
                        * np.cos(2 * math.pi * k[0] * x + ph[0])[None, None, :])
        return out

    rho = 1.0 + amp_rho * field()
    vel = [amp_u * field() for _ in range(3)]
    pp = amp_p * field()
    Q = np.empty((5, nz, ny, nx))
    Q[0] = rho
    for d in range(3):
        Q[1 + d] = rho * vel[d]
    Q[4] = pp / (params["gamma"] - 1.0) + 0.5 * rho * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)
    return Q
