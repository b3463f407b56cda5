"""FP64 CPU oracle: the frequency/time hybrid method, step by step.

TEST INFRASTRUCTURE ONLY -- imported by tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.

Each function follows one step of Anderson, Bruno & Lyon, "High-order,
dispersionless Fast-Hybrid wave equation solver, Part I" (arXiv 1807.02718),
cited by section and equation label.  Bessel functions come from
scipy.special, LU from LAPACK (scipy.linalg), the DFT is a direct O(M^2) sum
and the sinc is numpy.sinc.  Nothing is blocked, fused or reordered beyond
what the cited definitions state.

Readings of passages the paper leaves open:
  * frequencies omega_j = j W / F, j = 1..F; DFT grid of 2F points on [-W, W)
  * coupling eta = max(kappa, 1); wave speed c = 1 unless given
  * incident field u_inc = f(t - p.r/c), so the boundary signal is a = -f
  * V(r, 0) := 1 for plane-wave data (low-frequency limit), 0 for point sources
  * window centers s_k = 1.5 H (k - 1) for all integers k
  * active windows A(t) = {k : |t - s_k - tau0| <= pi / d_omega}
  * extra recentering shift tau0 (tau0 = 0 is the paper's choice)
  * sinc is the normalized sinc sin(pi x)/(pi x)
"""
from __future__ import annotations

import math
import numpy as np
from scipy import special, linalg

__all__ = [
    "frequency_grid", "curve_length", "discretization_sizes", "coupling",
    "geometry", "kress_weights", "kress_log_table", "assemble",
    "rhs_plane_wave", "rhs_point_source", "solve_density", "field",
    "field_full_grid", "eta_window", "window", "window_center",
    "window_indices", "window_spectra", "fourier_coefficients",
    "active_windows", "synthesize", "run", "curve_eval",
    "scaled_convolution_fast", "synthesize_uniform",
    "graded_mesh", "clenshaw_curtis_nodes", "lowfreq_frequencies", "chebyshev_moments",
    "fcc_integral", "gram_basis", "fc_gram_tables", "fc_continuation", "fc_coefficients",
    "fc_integral", "synthesize_lowfreq", "boundary_window_transforms", "synthesize_windowed",
    "synthesize_lowfreq_windowed", "assemble_dirichlet", "field_dirichlet", "run_general",
]


# ---------------------------------------------------------------------------
# O1. Frequency grid, discretization sizes, coupling parameter
# ---------------------------------------------------------------------------
def frequency_grid(W: float, F: int, c: float = 1.0):
    """Solve frequencies omega_j = j W/F (j = 1..F) and wavenumbers
    kappa = omega/c (Sec. 2.1, linear dispersion relation kappa = omega/c;
    the F frequencies feed the 2F-point DFT grid of Sec. 4.1.1, eq. fourier_approx)."""
    dw = W / F
    omega = dw * np.arange(1, F + 1, dtype=np.float64)
    return omega, omega / c


def curve_eval(curve, s):
    """x(s), x'(s), x''(s) of a trigonometric-polynomial curve; shapes (len(s), 2)."""
    s = np.asarray(s, dtype=np.float64)
    d = np.arange(curve.degree + 1, dtype=np.float64)[:, None]
    C, S = np.cos(d * s[None, :]), np.sin(d * s[None, :])
    out = []
    for cc, ss in ((curve.cx, curve.sx), (curve.cy, curve.sy)):
        cc = np.asarray(cc, dtype=np.float64); ss = np.asarray(ss, dtype=np.float64)
        x = cc @ C + ss @ S
        dx = (cc * d[:, 0]) @ (-S) + (ss * d[:, 0]) @ C
        ddx = -(cc * d[:, 0] ** 2) @ C - (ss * d[:, 0] ** 2) @ S
        out.append((x, dx, ddx))
    X = np.stack([out[0][0], out[1][0]], axis=1)
    dX = np.stack([out[0][1], out[1][1]], axis=1)
    ddX = np.stack([out[0][2], out[1][2]], axis=1)
    return X, dX, ddX


def curve_length(curve, n_quad: int = 4096) -> float:
    """Perimeter by the trapezoidal rule on the periodic speed |x'(s)|."""
    s = 2 * np.pi * np.arange(n_quad) / n_quad
    _, dX, _ = curve_eval(curve, s)
    return float(2 * np.pi / n_quad * np.sum(np.hypot(dX[:, 0], dX[:, 1])))


def discretization_sizes(kappa, length, ppw, n_min, n_mult, n_cap):
    """N_j = max(n_min, ceil(ppw * L * kappa / (2 pi) / n_mult) * n_mult), capped
    at n_cap: a fixed number of points per wavelength over the curve."""
    kappa = np.asarray(kappa, dtype=np.float64)
    raw = ppw * length * kappa / (2 * np.pi)
    N = np.ceil(raw / n_mult).astype(np.int64) * n_mult
    return np.minimum(np.maximum(N, n_min), n_cap)


def coupling(kappa):
    """Coupling parameter eta of the combined field equation (eq. CFIE_direct);
    any real nonzero value gives unique solvability; we take max(kappa, 1)."""
    return np.maximum(np.asarray(kappa, dtype=np.float64), 1.0)


# ---------------------------------------------------------------------------
# O2. Boundary nodes (the set C of boundary points, Sec. 5)
# ---------------------------------------------------------------------------
def geometry(curve, N: int):
    """Nodes t_i = 2 pi i / N on [0, 2 pi) with x, x', x'', |x'| and the outward
    unit normal nu = (x2', -x1')/|x'| (counter-clockwise curve).

    Rejects a clockwise or degenerate curve (signed area <= 0 or |x'| = 0)."""
    t = 2 * np.pi * np.arange(N) / N
    X, dX, ddX = curve_eval(curve, t)
    speed = np.hypot(dX[:, 0], dX[:, 1])
    if np.any(speed == 0.0) or not np.all(np.isfinite(X)):
        raise ValueError("degenerate curve")
    area = 0.5 * np.sum(X[:, 0] * dX[:, 1] - X[:, 1] * dX[:, 0]) * (2 * np.pi / N)
    if area <= 0:
        raise ValueError("curve must be counter-clockwise with positive area")
    nu = np.stack([dX[:, 1], -dX[:, 0]], axis=1) / speed[:, None]
    return dict(t=t, x=X, dx=dX, ddx=ddX, speed=speed, nu=nu)


# ---------------------------------------------------------------------------
# O3. Kress product-quadrature weights for the logarithmic kernel part
#     (the 2D Nystrom method cited in Sec. 2.3: Colton & Kress, Sec. 3.5)
# ---------------------------------------------------------------------------
def kress_weights(N: int):
    """R_l, l = 0..N-1 (N = 2n): weights of the rule
        int_0^{2pi} log(4 sin^2((t_i - tau)/2)) f(tau) dtau ~= sum_j R_{(i-j) mod N} f(t_j),
    R_l = -(2 pi / n) sum_{m=1}^{n-1} cos(m l pi / n) / m - (-1)^l pi / n^2."""
    if N % 2:
        raise ValueError("N must be even")
    n = N // 2
    l = np.arange(N)[:, None].astype(np.float64)
    m = np.arange(1, n)[None, :].astype(np.float64)
    R = -(2 * np.pi / n) * np.sum(np.cos(m * l * np.pi / n) / m, axis=1)
    R -= ((-1.0) ** np.arange(N)) * np.pi / n ** 2
    return R


def kress_log_table(N: int):
    """Lambda_l = log(4 sin^2(l pi / N)) for l = 1..N-1 (entry 0 unused, set 0)."""
    l = np.arange(N)
    out = np.zeros(N)
    out[1:] = np.log(4 * np.sin(l[1:] * np.pi / N) ** 2)
    return out


# ---------------------------------------------------------------------------
# O4/O5. Nystrom matrix and right-hand side of the direct CFIE (eq. CFIE_direct)
# ---------------------------------------------------------------------------
def assemble(geom, kappa: float, eta: float):
    """A_ij for  (1/2) psi + K*psi - i eta S psi  on the parametrized nodes.

    Kernels (parameter t at the target i, tau at the source j), with
    G = (i/4) H0^(1)(kappa |x - y|) (Sec. 2.3), d = x_j - x_i, r = |d|:
      M  = (i/4) H0(kappa r)                       (single layer)
      L  = (i kappa / 4) H1(kappa r) (nu_i . d) / r  (normal derivative at target)
    split as K = K1 log(4 sin^2((t-tau)/2)) + K2 with
      M1 = -J0(kappa r)/(4 pi),  L1 = -(kappa/(4 pi)) J1(kappa r) (nu_i . d)/r,
    and diagonal limits
      M2_ii = i/4 - (gamma + log(kappa |x'_i| / 2))/(2 pi),  L1_ii = 0,
      L2_ii = nu_i . x''_i / (4 pi |x'_i|^2).
    A_ij = delta_ij / 2 + |x'_j| [ R_{i-j} (L1 - i eta M1) + (pi/n) (L2 - i eta M2) ].
    """
    x, nu, speed, ddx = geom["x"], geom["nu"], geom["speed"], geom["ddx"]
    N = len(speed)
    n = N // 2
    R = kress_weights(N)
    Lam = kress_log_table(N)
    i_idx = np.arange(N)[:, None]
    j_idx = np.arange(N)[None, :]
    lidx = (i_idx - j_idx) % N
    d = x[None, :, :] - x[:, None, :]                 # d[i, j] = x_j - x_i
    r = np.hypot(d[..., 0], d[..., 1])
    diag = np.eye(N, dtype=bool)
    r_safe = np.where(diag, 1.0, r)
    z = kappa * r_safe
    J0, Y0, J1, Y1 = special.j0(z), special.y0(z), special.j1(z), special.y1(z)
    nud = nu[:, None, 0] * d[..., 0] + nu[:, None, 1] * d[..., 1]   # nu_i . d_ij
    logt = Lam[lidx]
    M = 0.25j * (J0 + 1j * Y0)
    M1 = -J0 / (4 * np.pi)
    M2 = M - M1 * logt
    L = 0.25j * kappa * (J1 + 1j * Y1) * nud / r_safe
    L1 = -(kappa / (4 * np.pi)) * J1 * nud / r_safe
    L2 = L - L1 * logt
    euler = 0.57721566490153286061
    M1[diag] = -1.0 / (4 * np.pi)
    M2[diag] = 0.25j - (euler + np.log(kappa * speed / 2)) / (2 * np.pi)
    L1[diag] = 0.0
    L2[diag] = (nu[:, 0] * ddx[:, 0] + nu[:, 1] * ddx[:, 1]) / (4 * np.pi * speed ** 2)
    K1 = L1 - 1j * eta * M1
    K2 = L2 - 1j * eta * M2
    A = (R[lidx] * K1 + (np.pi / n) * K2) * speed[None, :]
    A[diag] += 0.5
    return A


def rhs_plane_wave(geom, kappa: float, eta: float, p):
    """g = dB/dn - i eta B with B = exp(i kappa p.x) (eq. CFIE_direct with the
    boundary data replaced by the plane wave, Sec. 3.2 / eq. psikslow_repr)."""
    x, nu = geom["x"], geom["nu"]
    phase = np.exp(1j * kappa * (x @ np.asarray(p, dtype=np.float64)))
    return 1j * (kappa * (nu @ np.asarray(p, dtype=np.float64)) - eta) * phase


def rhs_point_source(geom, kappa: float, eta: float, r0):
    """g for B = (i/4) H0(kappa |x - r0|), a source r0 outside the closed domain."""
    x, nu = geom["x"], geom["nu"]
    dd = x - np.asarray(r0, dtype=np.float64)[None, :]
    rho = np.hypot(dd[:, 0], dd[:, 1])
    B = 0.25j * special.hankel1(0, kappa * rho)
    dB = -0.25j * kappa * special.hankel1(1, kappa * rho) * np.sum(nu * dd, axis=1) / rho
    return dB - 1j * eta * B


# ---------------------------------------------------------------------------
# O6. Dense solve (step F3)
# ---------------------------------------------------------------------------
def solve_density(A, g):
    """psi = A^{-1} g by LAPACK LU with partial pivoting; returns (psi, relres)
    with relres = ||g - A psi||_2 / ||g||_2."""
    lu, piv = linalg.lu_factor(A, check_finite=True)
    psi = linalg.lu_solve((lu, piv), g)
    res = np.linalg.norm(g - A @ psi) / np.linalg.norm(g)
    return psi, float(res)


# ---------------------------------------------------------------------------
# O7. Field evaluation (eq. freq_domain_repr / Ukslow_repr, step F5)
# ---------------------------------------------------------------------------
def field(geom, psi, kappa: float, obs):
    """V(r) = int_Gamma psi G dsigma ~= (pi/n) sum_i (i/4) H0(kappa |r - x_i|) |x'_i| psi_i
    (trapezoidal rule in the parameter, valid for r away from Gamma)."""
    x, speed = geom["x"], geom["speed"]
    N = len(speed)
    obs = np.asarray(obs, dtype=np.float64)
    dd = obs[:, None, :] - x[None, :, :]
    rr = np.hypot(dd[..., 0], dd[..., 1])
    z = kappa * rr
    G = 0.25j * (special.j0(z) + 1j * special.y0(z))
    return (2 * np.pi / N) * (G * speed[None, :]) @ psi


def assemble_dirichlet(geom, kappa: float, eta: float):
    """A_ij for  (1/2) phi + K phi - i eta S phi  (the combined double- and
    single-layer potential u = int [dG/dnu_y - i eta G] phi dsigma_y for an
    exterior Dirichlet problem with arbitrary data, Colton & Kress Sec. 3.2,
    discretized by the same Kress split as assemble): the double-layer kernel
      L = (i kappa / 4) H1(kappa r) (nu_j . (x_i - x_j)) / r
    takes the source normal nu_j where the direct equation's adjoint kernel
    takes the target normal; L1 = -(kappa/(4 pi)) J1(kappa r) (nu_j . (x_i -
    x_j))/r, and the diagonal limits are those of assemble (L2_ii is the
    curvature term for both kernels)."""
    x, nu, speed, ddx = geom["x"], geom["nu"], geom["speed"], geom["ddx"]
    N = len(speed)
    n = N // 2
    R = kress_weights(N)
    Lam = kress_log_table(N)
    lidx = (np.arange(N)[:, None] - np.arange(N)[None, :]) % N
    d = x[None, :, :] - x[:, None, :]                 # d[i, j] = x_j - x_i
    r = np.hypot(d[..., 0], d[..., 1])
    diag = np.eye(N, dtype=bool)
    r_safe = np.where(diag, 1.0, r)
    z = kappa * r_safe
    J0, Y0, J1, Y1 = special.j0(z), special.y0(z), special.j1(z), special.y1(z)
    nud = -(nu[None, :, 0] * d[..., 0] + nu[None, :, 1] * d[..., 1])   # nu_j . (x_i - x_j)
    logt = Lam[lidx]
    M = 0.25j * (J0 + 1j * Y0)
    M1 = -J0 / (4 * np.pi)
    M2 = M - M1 * logt
    L = 0.25j * kappa * (J1 + 1j * Y1) * nud / r_safe
    L1 = -(kappa / (4 * np.pi)) * J1 * nud / r_safe
    L2 = L - L1 * logt
    M1[diag] = -1.0 / (4 * np.pi)
    M2[diag] = 0.25j - (0.57721566490153286061 + np.log(kappa * speed / 2)) / (2 * np.pi)
    L1[diag] = 0.0
    L2[diag] = (nu[:, 0] * ddx[:, 0] + nu[:, 1] * ddx[:, 1]) / (4 * np.pi * speed ** 2)
    A = (R[lidx] * (L1 - 1j * eta * M1) + (np.pi / n) * (L2 - 1j * eta * M2)) * speed[None, :]
    A[diag] += 0.5
    return A


def field_dirichlet(geom, phi, kappa: float, eta: float, obs):
    """U(r) = int [dG(r, y)/dnu_y - i eta G(r, y)] phi(y) dsigma_y by the
    trapezoidal rule in the parameter (r away from Gamma), G = (i/4) H0:
    (2 pi/N) sum_j |x'_j| [ (i kappa/4) H1(kappa rho) nu_j . (r - x_j)/rho
    + (eta/4) H0(kappa rho) ] phi_j,  rho = |r - x_j|."""
    x, nu, speed = geom["x"], geom["nu"], geom["speed"]
    N = len(speed)
    obs = np.asarray(obs, dtype=np.float64)
    dd = obs[:, None, :] - x[None, :, :]
    rho = np.hypot(dd[..., 0], dd[..., 1])
    z = kappa * rho
    H0 = special.j0(z) + 1j * special.y0(z)
    H1 = special.j1(z) + 1j * special.y1(z)
    dl = 0.25j * kappa * H1 * (nu[None, :, 0] * dd[..., 0] + nu[None, :, 1] * dd[..., 1]) / rho
    return (2 * np.pi / N) * ((dl + 0.25 * eta * H0) * speed[None, :]) @ phi


def field_full_grid(V_pos, zero_value):
    """Extend V(r, omega_j), j = 1..F, to the DFT grid omega_l = (l - F) d_omega,
    l = 0..2F-1, on [-W, W): V(r, -omega) = conj V(r, omega) (real time signals)
    and V(r, 0) = zero_value."""
    Nr, F = V_pos.shape
    out = np.zeros((Nr, 2 * F), dtype=np.complex128)
    out[:, F] = zero_value
    out[:, F + 1:] = V_pos[:, : F - 1]
    out[:, :F] = np.conj(V_pos[:, ::-1])
    return out


# ---------------------------------------------------------------------------
# O8. Partition of unity (Sec. 3.1, eq. window_func)
# ---------------------------------------------------------------------------
def eta_window(u):
    """eta(u) = exp(2 e^{-1/u} / (u - 1)) on (0, 1); eta = 1 for u <= 0, 0 for u >= 1."""
    u = np.asarray(u, dtype=np.float64)
    out = np.where(u <= 0.0, 1.0, 0.0)
    m = (u > 0.0) & (u < 1.0)
    um = u[m]
    out[m] = np.exp(2.0 * np.exp(-1.0 / um) / (um - 1.0))
    return out


def window(t, H: float):
    """w(t): 1 - eta((t+H)/(H/2)) on [-H, -H/2], 1 on (-H/2, H/2),
    eta((t - H/2)/(H/2)) on [H/2, H], 0 for |t| > H (eq. window_func)."""
    t = np.asarray(t, dtype=np.float64)
    out = np.zeros_like(t)
    left = (t >= -H) & (t <= -H / 2)
    mid = (t > -H / 2) & (t < H / 2)
    right = (t >= H / 2) & (t <= H)
    out[left] = 1.0 - eta_window((t[left] + H) / (H / 2))
    out[mid] = 1.0
    out[right] = eta_window((t[right] - H / 2) / (H / 2))
    return out


def window_center(k, H: float):
    """s_k = 3 (k - 1) H / 2 (Sec. 3.1)."""
    return 1.5 * H * (np.asarray(k, dtype=np.float64) - 1.0)


def window_indices(t_lo: float, t_hi: float, H: float):
    """All integers k whose support [s_k - H, s_k + H] meets [t_lo, t_hi]."""
    k_lo = math.floor((t_lo - H) / (1.5 * H)) + 1
    k_hi = math.ceil((t_hi + H) / (1.5 * H)) + 1
    ks = np.arange(k_lo - 1, k_hi + 2)
    s = window_center(ks, H)
    keep = (s + H >= t_lo) & (s - H <= t_hi)
    return ks[keep]


# ---------------------------------------------------------------------------
# O9. Windowed, recentered signal spectra (eq. Bkslow_eqn, steps F1-F2)
# ---------------------------------------------------------------------------
def window_spectra(signal, H: float, ks, omega_l):
    """B_k^slow(omega_l) = int a_k(t + s_k) e^{i omega t} dt with a_k = w_k a and
    a = -f (sound-soft data b = -u_inc), by the rectangle/trapezoidal rule on the
    signal samples (the integrand vanishes with all derivatives at the ends)."""
    t = signal.t
    a = -np.asarray(signal.f, dtype=np.float64)
    out = np.zeros((len(ks), len(omega_l)), dtype=np.complex128)
    for i, k in enumerate(ks):
        sk = window_center(k, H)
        tau = t - sk
        wk = window(tau, H)
        sel = wk != 0.0
        out[i] = signal.dt * (np.exp(1j * np.outer(omega_l, tau[sel])) @ (wk[sel] * a[sel]))
    return out


# ---------------------------------------------------------------------------
# O10. Fourier-series coefficients on [-W, W) (eq. fourier_approx, DFT case)
# ---------------------------------------------------------------------------
def fourier_coefficients(G, W: float):
    """c_m, m = -F..F-1, of G(omega) ~= sum_m c_m e^{i pi m omega / W} from the
    2F samples G(omega_l), omega_l = -W + l W/F: direct DFT sum
    c_m = (1/2F) sum_l G_l e^{-i pi m omega_l / W}.  G has shape (..., 2F)."""
    M = G.shape[-1]
    F = M // 2
    dw = W / F
    omega_l = -W + dw * np.arange(M)
    m = np.arange(-F, F)
    E = np.exp(-1j * np.pi * np.outer(omega_l, m) / W)      # (2F, 2F)
    return (G @ E) / M


# ---------------------------------------------------------------------------
# O11. Scaled-convolution synthesis and sum over windows (eqs. approx,
#      discConv, ukW, uk_def, final_u; steps T1a, T2, T5)
# ---------------------------------------------------------------------------
def active_windows(t: float, ks, H: float, tau0: float, dw: float):
    s = window_center(ks, H)
    return np.abs(t - s - tau0) <= np.pi / dw


def synthesize(V_full, Bslow, ks, H, tau0, W, times, track_tol=0.0):
    """u(r, t) = sum_{k in A(t)} u_k^{W,J}(r, t) with
        u_k(r, t) = (1/2pi) int_{-W}^{W} B_k^slow(w) V(r, w) e^{-i w (t - s_k)} dw
                  = Re (W/pi) sum_m c_{k,m}(r) sinc(W (t - s_k - tau0)/pi - m),
    c_{k,m}(r) the Fourier coefficients of B_k^slow V e^{-i w tau0} on [-W, W).
    track_tol > 0: active-partition tracking (Sec. 3.2, remark on tracking:
    a partition enters a region only where it exceeds a tolerance there).
    Partition k is left out everywhere when its spectrum is negligible,
    max_l (|Re B_k| + |Im B_k|) <= track_tol times the largest such maximum
    (then |u_k| <= (W/pi) 2F max_l |B_k| max_l |V(r, .)|), and at point r
    when b_k(r) = sum_m |Re c_{k,m}(r)|, which bounds |u_k(r, .)| / (W/pi)
    since |sinc| <= 1, is at most track_tol times the largest b over the
    remaining partitions; only partitions active at some sample time count.
    Returns (u, max |Im|) where Im is the imaginary part before taking Re."""
    Nr, M = V_full.shape
    F = M // 2
    dw = W / F
    omega_l = -W + dw * np.arange(M)
    m = np.arange(-F, F)
    times = np.asarray(times)
    u = np.zeros((Nr, len(times)))
    im_max = 0.0
    shift = np.exp(-1j * omega_l * tau0)
    parts = []
    for ik, k in enumerate(ks):
        sk = window_center(k, H)
        act = np.abs(times - sk - tau0) <= np.pi / dw
        if not np.any(act):
            continue
        G = Bslow[ik][None, :] * V_full * shift[None, :]
        c = fourier_coefficients(G, W)                        # (Nr, 2F)
        wmax = float(np.max(np.abs(Bslow[ik].real) + np.abs(Bslow[ik].imag)))
        parts.append((sk, act, c, np.sum(np.abs(c.real), axis=1), wmax))
    if track_tol > 0:
        wcut = track_tol * max((w for *_, w in parts), default=0.0)
        parts = [pt for pt in parts if pt[4] > wcut]
    cut = track_tol * max((float(np.max(pt[3])) for pt in parts), default=0.0) if track_tol > 0 else -1.0
    for sk, act, c, b, _ in parts:
        keep = b > cut
        tt = times[act]
        S = np.sinc(W * (tt[None, :] - sk - tau0) / np.pi - m[:, None])   # (2F, nt)
        uk = (W / np.pi) * (c @ S)
        im_max = max(im_max, float(np.max(np.abs(uk.imag))) if uk.size else 0.0)
        u[np.ix_(keep, act)] += uk.real[keep]
    return u, im_max


# ---------------------------------------------------------------------------
# O12. Fast scaled convolution for uniform time grids (Sec. 4.1.2, FFT
#      accelerated evaluation of scaled discrete convolutions:
#      eqs. conv_sum, approx_conv_sum; Table 1)
# ---------------------------------------------------------------------------
def scaled_convolution_fast(a, x, L: int):
    """Approximation of d(x) = sum_m a_m b(x - m), m = -M/2..M/2-1, with the
    kernel b(q) = sinc(q) of eq. discConv (there 2A = P: the coefficients span
    the whole period), by eq. approx_conv_sum with gamma = 1:
        d(x) ~= (1/L) sum_{p=-L/2}^{L/2-1} C_p B_p e^{2 pi i p x / L},
        C_p = sum_m a_m e^{-2 pi i m p / L},
        B_p = sum_{q=-L/2}^{L/2-1} b(q) e^{-2 pi i q p / L},
    that is, b replaced by its L-periodic trigonometric interpolant on the
    integers, evaluated at the real arguments x - m (the paper's beta n - m on
    a uniform grid).  Each sum is written out as a matrix product; no FFT.
    a: shape (..., M), real or complex; x: the real arguments, shape (n,).
    Returns the real part, shape (..., n)."""
    M = a.shape[-1]
    m = np.arange(-(M // 2), M // 2)
    p = np.arange(-(L // 2), L // 2)
    q = p
    C = a @ np.exp(-2j * np.pi * np.outer(m, p) / L)
    B = np.sinc(q) @ np.exp(-2j * np.pi * np.outer(q, p) / L)
    E = np.exp(2j * np.pi * np.outer(p, np.asarray(x, dtype=np.float64)) / L)
    return ((C * B) @ E).real / L


def synthesize_uniform(V_full, Bslow, ks, H, tau0, W, t_first, t_step, n_t, L: int, t_index=None,
                       track_tol=0.0):
    """u(r, t_n) on the uniform grid t_n = t_first + n t_step, n < n_t, as
    synthesize (same windows, coefficients, active sets and tracking rules)
    with each window's sum over m, sum_m Re c_{k,m} sinc(x - m), x = W (t_n -
    s_k - tau0)/pi, replaced by scaled_convolution_fast of size L.  t_index:
    only these grid indices (columns of the result, in the given order)."""
    Nr, M = V_full.shape
    F = M // 2
    dw = W / F
    omega_l = -W + dw * np.arange(M)
    times = t_first + t_step * np.arange(n_t)
    if t_index is not None:
        times = times[np.asarray(t_index)]
    u = np.zeros((Nr, len(times)))
    shift = np.exp(-1j * omega_l * tau0)
    parts = []
    for ik, k in enumerate(ks):
        sk = window_center(k, H)
        act = np.abs(times - sk - tau0) <= np.pi / dw
        if not np.any(act):
            continue
        G = Bslow[ik][None, :] * V_full * shift[None, :]
        a = fourier_coefficients(G, W).real
        wmax = float(np.max(np.abs(Bslow[ik].real) + np.abs(Bslow[ik].imag)))
        parts.append((sk, act, a, np.sum(np.abs(a), axis=1), wmax))
    if track_tol > 0:
        wcut = track_tol * max((w for *_, w in parts), default=0.0)
        parts = [pt for pt in parts if pt[4] > wcut]
    cut = track_tol * max((float(np.max(pt[3])) for pt in parts), default=0.0) if track_tol > 0 else -1.0
    for sk, act, a, b, _ in parts:
        keep = b > cut
        idx = np.nonzero(act)[0]
        x = W * (times[idx] - sk - tau0) / np.pi
        u[np.ix_(keep, idx)] += (W / np.pi) * scaled_convolution_fast(a[keep], x, L)
    return u


# ---------------------------------------------------------------------------
# O13. Low-frequency singular quadrature for 2D (Sec. 4.2, eqs.
#      fourier_sing_decomp, gradedmesh, gradedmeshIntRule) with Fourier
#      continuation of the smooth part (Sec. 4.1.1, Remark Fourier-FC;
#      steps T1b, T2b-T2d)
# ---------------------------------------------------------------------------
def graded_mesh(omega_c: float, M: int, q: float):
    """mu_j = omega_c (j / M)^q, j = 0..M (eq. gradedmesh; mu_0 = 0 is kept, so
    that the composite rule covers all of (0, omega_c])."""
    return omega_c * (np.arange(M + 1, dtype=np.float64) / M) ** q


def clenshaw_curtis_nodes(a: float, b: float, n: int):
    """The n + 1 Clenshaw-Curtis (Chebyshev extreme) points of [a, b],
    (a + b)/2 + (b - a)/2 cos(pi i / n), i = 0..n (descending)."""
    return 0.5 * (a + b) + 0.5 * (b - a) * np.cos(np.pi * np.arange(n + 1) / n)


def lowfreq_frequencies(W: float, F: int, jc: int, M: int, n: int, q: float):
    """The frequency sets of the 2D method (Sec. 5, F = F^smooth U F^sing):
    omega_c = jc W / F; F^smooth = the solve grid on [omega_c, W], omega_c +
    i W / F, i = 0..F - jc; F^sing = the Clenshaw-Curtis points of the M
    subintervals [mu_{j-1}, mu_j] of the graded mesh, n + 1 per subinterval.
    Returns (omega_c, smooth grid, mu, nodes[M][n + 1])."""
    h = W / F
    omega_c = jc * h
    smooth = omega_c + h * np.arange(F - jc + 1)
    mu = graded_mesh(omega_c, M, q)
    nodes = [clenshaw_curtis_nodes(mu[j], mu[j + 1], n) for j in range(M)]
    return omega_c, smooth, mu, nodes


def chebyshev_moments(n: int, kappa: float):
    """m_k = int_{-1}^{1} T_k(x) e^{-i kappa x} dx, k = 0..n (the modified
    moments of the Filon-Clenshaw-Curtis rule), by Gauss-Legendre quadrature
    with enough nodes (64 + 3|kappa|/4) that the entire integrand is
    integrated to rounding."""
    ng = 64 + int(np.ceil(0.75 * abs(kappa)))
    x, w = np.polynomial.legendre.leggauss(ng)
    T = np.cos(np.arange(n + 1)[:, None] * np.arccos(np.clip(x, -1.0, 1.0))[None, :])
    return T @ (w * np.exp(-1j * kappa * x))


def fcc_integral(values, a: float, b: float, n: int, t):
    """Filon-Clenshaw-Curtis rule (Sec. 4.2): int_a^b Q_n F(w) e^{-i w t} dw,
    Q_n F the degree-n polynomial interpolating F at the Clenshaw-Curtis points
    of [a, b] (values in the order of clenshaw_curtis_nodes).  The interpolant
    is written in Chebyshev form, p = sum_k alpha_k T_k(x), w = (a+b)/2 +
    (b-a)/2 x, by solving the interpolation conditions; each moment is exact
    (chebyshev_moments).  t: array of times."""
    x = np.cos(np.pi * np.arange(n + 1) / n)
    T = np.cos(np.outer(np.arccos(x), np.arange(n + 1)))
    alpha = np.linalg.solve(T, np.asarray(values, dtype=np.complex128))
    rho, delta = 0.5 * (b - a), 0.5 * (a + b)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    return np.array([rho * np.exp(-1j * delta * tt) * (alpha @ chebyshev_moments(n, rho * tt)) for tt in t])


def gram_basis(d: int):
    """Gram polynomials on the d points 0, 1, .., d-1: the columns of Q (d x d,
    values at the points) are orthonormal in the discrete inner product, the
    k-th of degree k; G_k(x) = sum_l R^{-1}[l, k] x^l.  High precision
    (mpmath, 60 digits); returns (Q as float64, R^{-1} as mpmath matrix)."""
    import mpmath as mp
    with mp.workdps(60):
        Vm = mp.matrix(d, d)
        for j in range(d):
            for l in range(d):
                Vm[j, l] = mp.mpf(j) ** l
        Q, R = mp.qr(Vm)
        # sign convention: positive leading coefficient of every G_k
        for k in range(d):
            if R[k, k] < 0:
                for j in range(d):
                    Q[j, k] = -Q[j, k]
                for l in range(d):
                    R[k, l] = -R[k, l]
        Rinv = R ** -1
        Qf = np.array([[float(Q[i, j]) for j in range(d)] for i in range(d)])
    return Qf, Rinv


_FC_CACHE = {}


def fc_gram_tables(d: int = 10, C: int = 25, oversample: int = 10):
    """FC(Gram) continuation tables (Remark Fourier-FC; the FC(Gram) Fourier
    continuation cited there).  For each Gram polynomial G_k, its "blend to
    zero" extension: the trigonometric polynomial phi_k of period 2 (d + C)
    and degree d + C (in the grid unit), least-squares closest to G_k on [0,
    d - 1] and to 0 on [d + C, 2d + C - 1], both sampled `oversample` times
    per unit; A[c, k] = phi_k(d + c), c = 0..C-1.  Full-rank least squares
    solved in 45-digit arithmetic (mpmath SVD).  Returns (A [C, d], Q [d, d])
    as float64, cached per (d, C, oversample)."""
    key = (d, C, oversample)
    if key in _FC_CACHE:
        return _FC_CACHE[key]
    import mpmath as mp
    Qf, Rinv = gram_basis(d)
    with mp.workdps(100):
        P = 2 * (d + C)
        B = d + C
        xm = [mp.mpf(i) / oversample for i in range((d - 1) * oversample + 1)]
        xz = [mp.mpf(d + C) + mp.mpf(i) / oversample for i in range((d - 1) * oversample + 1)]

        def basis(x):
            row = [mp.mpf(1)]
            for m in range(1, B + 1):
                row += [mp.cos(2 * mp.pi * m * x / P), mp.sin(2 * mp.pi * m * x / P)]
            return row

        # normal equations of the full-rank least-squares problem, in 100
        # digits (its condition number squared is about 1e48 for d = 10)
        Mm = mp.matrix([basis(x) for x in xm])
        Mz = mp.matrix([basis(x) for x in xz])
        G = Mm.T * Mm + Mz.T * Mz
        Ginv = G ** -1
        Ec = mp.matrix([basis(mp.mpf(d + c)) for c in range(C)])
        A = np.zeros((C, d))
        for k in range(d):
            y = mp.matrix([sum(Rinv[l, k] * x ** l for l in range(d)) for x in xm])
            coef = Ginv * (Mm.T * y)
            vals = Ec * coef
            A[:, k] = [float(vals[c]) for c in range(C)]
    _FC_CACHE[key] = (A, Qf)
    return A, Qf


def fc_continuation(f, A, Q):
    """The FC(Gram) periodic extension of n samples f (n >= d) of a smooth,
    non-periodic function on an equispaced grid: the n samples followed by C
    continuation values, the blend to zero of the last d samples' Gram
    projection plus the blend from zero (mirrored) of the first d samples'.
    Returns the n + C values of one period."""
    f = np.asarray(f, dtype=np.complex128)
    n = len(f)
    C, d = A.shape
    g = np.zeros(n + C, dtype=np.complex128)
    g[:n] = f
    g[n:] += A @ (Q.T @ f[n - d:])
    g[n:] += (A @ (Q.T @ f[:d][::-1]))[::-1]
    return g


def fc_coefficients(f, A, Q):
    """Coefficients c_m, m = -L/2..L/2-1 (L = n + C, index m + L/2), of the
    trigonometric polynomial of period L h interpolating the FC(Gram)
    extension (eq. fourier_approx with P = L h != 2A): direct DFT sum."""
    g = fc_continuation(f, A, Q)
    L = len(g)
    m = np.arange(-(L // 2), L - L // 2)
    jj = np.arange(L)
    return (np.exp(-2j * np.pi * np.outer(m, jj) / L) @ g) / L


def fc_integral(c, omega_a: float, h: float, n: int, t):
    """int_{omega_a}^{omega_a + (n-1) h} sum_m c_m e^{2 pi i m (w - omega_a)/P}
    e^{-i w t} dw, P = L h: term-wise exact integration (eq. approx with
    A = (n - 1) h / 2, P != 2A), written with the normalized sinc."""
    L = len(c)
    P = L * h
    D = (n - 1) * h
    m = np.arange(-(L // 2), L - L // 2)
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    nu = 2 * np.pi * m[None, :] / P - t[:, None]
    ker = np.exp(0.5j * nu * D) * D * np.sinc(nu * D / (2 * np.pi))
    return np.exp(-1j * omega_a * t) * (ker @ c)


def synthesize_lowfreq(V_full, V_sing, signal, H, tau0, W, F, jc, M, n, q, times, fc_d=10, fc_C=25):
    """Time samples by the 2D low-frequency decomposition (eq.
    fourier_sing_decomp; steps T1b, T2b-T2d, T5): for every window k whose
    support meets the signal's range and every point r,
        u_k(r, t) = (1/pi) Re [ I_0(t') + I_+(t') ],  t' = t - s_k - tau0,
    with F_k(w) = B_k^slow(w) V(r, w) e^{-i w tau0}; I_+ = int_{omega_c}^{W}
    F_k e^{-i w t'} dw from the FC(Gram) continuation of F_k on the grid of
    [omega_c, W] (fc_coefficients, fc_integral), I_0 = int_0^{omega_c} by the
    composite Filon-Clenshaw-Curtis rule on the graded mesh (eq.
    gradedmeshIntRule, fcc_integral); the negative frequencies enter as the
    complex conjugate (real signals), hence (1/2 pi) 2 Re.  Every window with
    signal content is summed at every time (in 2D the low-frequency part of
    u_k decays only algebraically in time).
    V_full: [Nr][2F] on the DFT grid (as field_full_grid); V_sing: [Nr][M][n+1]
    at the nodes of lowfreq_frequencies."""
    omega_c, smooth, mu, nodes = lowfreq_frequencies(W, F, jc, M, n, q)
    A, Q = fc_gram_tables(fc_d, fc_C)
    Nr = V_full.shape[0]
    # V at the smooth grid: omega = (jc + i) W/F -> index F + jc + i; +W only as conj at index 0
    idx = F + jc + np.arange(F - jc + 1)
    Vs = np.empty((Nr, len(smooth)), dtype=np.complex128)
    inside = idx < 2 * F
    Vs[:, inside] = V_full[:, idx[inside]]
    Vs[:, ~inside] = np.conj(V_full[:, 0])[:, None]
    times = np.asarray(times, dtype=np.float64)
    u = np.zeros((Nr, len(times)))
    ks = window_indices(signal.t[0], signal.t[-1], H)
    for k in ks:
        sk = window_center(k, H)
        tp = times - sk - tau0
        Bs = window_spectra(signal, H, [k], smooth)[0] * np.exp(-1j * smooth * tau0)
        Bn = [window_spectra(signal, H, [k], nodes[j])[0] * np.exp(-1j * nodes[j] * tau0) for j in range(M)]
        for r in range(Nr):
            c = fc_coefficients(Bs * Vs[r], A, Q)
            I = fc_integral(c, omega_c, W / F, len(smooth), tp)
            for j in range(M):
                I = I + fcc_integral(Bn[j] * V_sing[r, j], mu[j], mu[j + 1], n, tp)
            u[r] += I.real / np.pi
    return u


# ---------------------------------------------------------------------------
# O14. General incident fields (eq. bkdef2): windowed boundary data per node
# ---------------------------------------------------------------------------
def boundary_window_transforms(samples, t0, dt, H, ks, omega):
    """The recentred transforms of the windowed boundary data of eq. bkdef2,
        B_k(x_i, w) = int w(t) b(x_i, t + s_k) e^{i w t} dt,
    by the rectangle rule on the samples b(x_i, t0 + n dt) (the integrand
    vanishes with all derivatives at the ends), for windows ks and
    frequencies omega.  samples: [N][n_t] real.  Returns [K][F][N] complex."""
    samples = np.asarray(samples, dtype=np.float64)
    t = t0 + dt * np.arange(samples.shape[1])
    out = np.zeros((len(ks), len(omega), samples.shape[0]), dtype=np.complex128)
    for q, k in enumerate(ks):
        tau = t - window_center(k, H)
        wk = window(tau, H)
        sel = wk != 0.0
        out[q] = dt * (np.exp(1j * np.outer(omega, tau[sel])) @ (wk[sel][:, None] * samples[:, sel].T))
    return out


def synthesize_windowed(V_k, ks, H, tau0, W, times):
    """u(r, t) = sum_{k in A(t)} Re (W/pi) sum_m c_{k,m}(r) sinc(W (t - s_k -
    tau0)/pi - m) with c_{k,m}(r) the Fourier coefficients of U_k^slow(r, w)
    e^{-i w tau0} on [-W, W): the synthesis of synthesize with each window's
    own frequency-domain field (the windowed boundary data already inside it)
    instead of B_k^slow(w) V(r, w).  V_k: [K][Nr][2F] on the DFT grid."""
    K, Nr, M = V_k.shape
    F = M // 2
    dw = W / F
    omega_l = -W + dw * np.arange(M)
    m = np.arange(-F, F)
    times = np.asarray(times)
    u = np.zeros((Nr, len(times)))
    shift = np.exp(-1j * omega_l * tau0)
    for q, k in enumerate(ks):
        sk = window_center(k, H)
        act = np.abs(times - sk - tau0) <= np.pi / dw
        if not np.any(act):
            continue
        c = fourier_coefficients(V_k[q] * shift[None, :], W)
        S = np.sinc(W * (times[act][None, :] - sk - tau0) / np.pi - m[:, None])
        u[:, act] += ((W / np.pi) * (c @ S)).real
    return u


def synthesize_lowfreq_windowed(V_k, V_k_sing, ks, H, tau0, W, F, jc, M, n, q, times, fc_d=10, fc_C=25):
    """synthesize_lowfreq with each window's own field (general boundary
    data): F_k(w) = V_k(r, w) e^{-i w tau0} (the windowed data already inside
    V_k, no spectrum factor), I_+ from its FC(Gram) continuation on the grid
    of [omega_c, W] and I_0 by the graded Filon-Clenshaw-Curtis rule, summed
    over all windows at every time.  V_k: [K][Nr][2F] on the DFT grid;
    V_k_sing: [K][Nr][M][n+1] at the nodes of lowfreq_frequencies."""
    omega_c, smooth, mu, nodes = lowfreq_frequencies(W, F, jc, M, n, q)
    A, Q = fc_gram_tables(fc_d, fc_C)
    K, Nr = V_k.shape[0], V_k.shape[1]
    idx = F + jc + np.arange(F - jc + 1)
    inside = idx < 2 * F
    times = np.asarray(times, dtype=np.float64)
    u = np.zeros((Nr, len(times)))
    es = np.exp(-1j * smooth * tau0)
    en = [np.exp(-1j * nodes[j] * tau0) for j in range(M)]
    for qw, k in enumerate(ks):
        tp = times - window_center(k, H) - tau0
        Vs = np.empty((Nr, len(smooth)), dtype=np.complex128)
        Vs[:, inside] = V_k[qw][:, idx[inside]]
        Vs[:, ~inside] = np.conj(V_k[qw][:, 0])[:, None]
        for r in range(Nr):
            c = fc_coefficients(es * Vs[r], A, Q)
            I = fc_integral(c, omega_c, W / F, len(smooth), tp)
            for j in range(M):
                I = I + fcc_integral(en[j] * V_k_sing[qw, r, j], mu[j], mu[j + 1], n, tp)
            u[r] += I.real / np.pi
    return u


def run_general(curve, W, F, N, b, t0, dt, H, tau0, obs, times, c=1.0, lowfreq=None):
    """The whole path for a general incident field (eq. bkdef2): Dirichlet
    data b(x_i, t) = -u_inc sampled at the N nodes (fixed N at every
    frequency); per window k the recentred transforms B_k at every solve
    frequency, the exterior Dirichlet problem with data B_k by the combined
    potential (assemble_dirichlet, field_dirichlet: the windowed data w_k b
    are not the trace of a wave, so the direct equation's right-hand side
    does not apply to them), and the synthesis of every window's own field
    (synthesize_windowed).  The zero-frequency sample of each window's field
    is taken as 0.  lowfreq = dict(jc, M, n, q): the same at the graded
    Clenshaw-Curtis frequencies too, synthesized by
    synthesize_lowfreq_windowed (the value at omega = 0, the first node,
    again 0: it enters the rule only through the first subinterval, of width
    mu_1 ~ 1e-11 omega_c).  b: [N][n_t].  Returns (u, ks)."""
    gm = geometry(curve, N)
    t_hi = t0 + dt * (np.asarray(b).shape[1] - 1)
    ks = window_indices(t0, t_hi, H)

    def window_fields(om):
        """V_k(r, om) for every window, [K][Nr][len(om)] (0 at om = 0)."""
        ka = np.asarray(om) / c
        et = coupling(np.where(ka > 0, ka, 1.0))
        Bk = boundary_window_transforms(b, t0, dt, H, ks, om)
        out = np.zeros((len(ks), len(obs), len(om)), dtype=np.complex128)
        for j in range(len(om)):
            if ka[j] == 0.0:
                continue
            lu = linalg.lu_factor(assemble_dirichlet(gm, ka[j], et[j]))
            for qw in range(len(ks)):
                out[qw, :, j] = field_dirichlet(gm, linalg.lu_solve(lu, Bk[qw, j]), ka[j], et[j], obs)
        return out

    omega, _ = frequency_grid(W, F, c)
    Vg = window_fields(omega)
    V_k = np.zeros((len(ks), len(obs), 2 * F), dtype=np.complex128)
    V_k[:, :, F + 1:] = Vg[:, :, : F - 1]
    V_k[:, :, :F] = np.conj(Vg[:, :, ::-1])
    if lowfreq is None:
        return synthesize_windowed(V_k, ks, H, tau0, W, times), ks
    jc, M, n, q = lowfreq["jc"], lowfreq["M"], lowfreq["n"], lowfreq["q"]
    _, _, _, nodes = lowfreq_frequencies(W, F, jc, M, n, q)
    Vn = window_fields(np.concatenate(nodes))
    V_sing = Vn.reshape(len(ks), len(obs), M, n + 1)
    return synthesize_lowfreq_windowed(V_k, V_sing, ks, H, tau0, W, F, jc, M, n, q, times), ks


# ---------------------------------------------------------------------------
# Whole pipeline (F1-F5, T0-T6)
# ---------------------------------------------------------------------------
def run(curve, W, F, N_rule, direction, signal, H, tau0, obs, times, c=1.0,
        incidence="plane", r0=None, return_all=False, lowfreq=None):
    """Scattered field u(r, t) on obs x times.  N_rule is an int (fixed N) or a
    dict(ppw, n_min, n_mult, n_cap).  lowfreq = dict(jc, M, n, q) selects the
    2D low-frequency decomposition (synthesize_lowfreq), with the extra
    frequency solves at the graded Clenshaw-Curtis points."""
    omega, kappa = frequency_grid(W, F, c)
    if isinstance(N_rule, dict):
        Ns = discretization_sizes(kappa, curve_length(curve), **N_rule)
    else:
        Ns = np.full(F, int(N_rule))
    eta = coupling(kappa)
    geoms = {}
    psis, res = [], []
    Vpos = np.zeros((len(obs), F), dtype=np.complex128)
    for j in range(F):
        N = int(Ns[j])
        if N not in geoms:
            geoms[N] = geometry(curve, N)
        gm = geoms[N]
        A = assemble(gm, kappa[j], eta[j])
        if incidence == "plane":
            g = rhs_plane_wave(gm, kappa[j], eta[j], direction)
        else:
            g = rhs_point_source(gm, kappa[j], eta[j], r0)
        psi, rr = solve_density(A, g)
        psis.append(psi); res.append(rr)
        Vpos[:, j] = field(gm, psi, kappa[j], obs)
    V_full = field_full_grid(Vpos, 1.0 if incidence == "plane" else 0.0)
    if lowfreq is not None:
        lf = dict(lowfreq)
        omega_c, _, _, nodes = lowfreq_frequencies(W, F, lf["jc"], lf["M"], lf["n"], lf["q"])
        zero = 1.0 if incidence == "plane" else 0.0
        V_sing = np.zeros((len(obs), lf["M"], lf["n"] + 1), dtype=np.complex128)
        for jm in range(lf["M"]):
            for i, om in enumerate(nodes[jm]):
                if om == 0.0:
                    V_sing[:, jm, i] = zero
                    continue
                kap = om / c
                if isinstance(N_rule, dict):
                    N = int(discretization_sizes([kap], curve_length(curve), **N_rule)[0])
                else:
                    N = int(N_rule)
                if N not in geoms:
                    geoms[N] = geometry(curve, N)
                gm = geoms[N]
                et = float(coupling(kap))
                A = assemble(gm, kap, et)
                g = rhs_plane_wave(gm, kap, et, direction) if incidence == "plane" else \
                    rhs_point_source(gm, kap, et, r0)
                psi, _ = solve_density(A, g)
                V_sing[:, jm, i] = field(gm, psi, kap, obs)
        u = synthesize_lowfreq(V_full, V_sing, signal, H, tau0, W, F, lf["jc"], lf["M"], lf["n"], lf["q"], times)
        if return_all:
            return dict(u=u, psi=psis, res=res, Vpos=Vpos, V=V_full, V_sing=V_sing, Ns=Ns, kappa=kappa, eta=eta)
        return u
    dw = W / F
    omega_l = -W + dw * np.arange(2 * F)
    t = signal.t
    ks = window_indices(t[0], t[-1], H)
    act_any = np.zeros(len(ks), dtype=bool)
    for tt in np.asarray(times):
        act_any |= active_windows(tt, ks, H, tau0, dw)
    ks = ks[act_any]
    B = window_spectra(signal, H, ks, omega_l)
    u, im_max = synthesize(V_full, B, ks, H, tau0, W, times)
    if return_all:
        return dict(u=u, im_max=im_max, psi=psis, res=res, Vpos=Vpos, V=V_full,
                    ks=ks, B=B, Ns=Ns, kappa=kappa, eta=eta)
    return u
