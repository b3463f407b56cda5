"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds input data only (curves, incident signals, observation
points, sample times and the parameter sets that name a workload).  It holds
none of the solver's arithmetic: no quadrature, no Green's function, no
window function, no discretization rule.  Both the CPU oracle and the GPU
path take what it returns as plain arrays.

Curves are real trigonometric polynomials in the parameter s in [0, 2*pi):

    x1(s) = sum_d cx[d] cos(d s) + sx[d] sin(d s)
    x2(s) = sum_d cy[d] cos(d s) + sy[d] sin(d s)

traversed counter-clockwise.  Signals are uniform samples f(t0 + n dt) of a
compactly supported incident time signal; the incident field is
u_inc(r, t) = f(t - p.r / c).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np


# --------------------------------------------------------------------------
# Curves
# --------------------------------------------------------------------------
@dataclass
class Curve:
    """Trigonometric-polynomial curve; arrays have length degree + 1."""
    name: str
    cx: np.ndarray
    sx: np.ndarray
    cy: np.ndarray
    sy: np.ndarray

    @property
    def degree(self) -> int:
        return len(self.cx) - 1


def _pad(a, n):
    out = np.zeros(n)
    out[: len(a)] = a
    return out


def circle(radius: float = 1.0, center=(0.0, 0.0)) -> Curve:
    """Circle of the given radius, x = c + R (cos s, sin s)."""
    return Curve("circle",
                 np.array([center[0], radius]), np.array([0.0, 0.0]),
                 np.array([center[1], 0.0]), np.array([0.0, radius]))


def kite() -> Curve:
    """Kite x = (cos s + 0.65 cos 2s - 0.65, 1.5 sin s) (Sec. 6.2 of the paper)."""
    return Curve("kite",
                 np.array([-0.65, 1.0, 0.65]), np.zeros(3),
                 np.zeros(3), np.array([0.0, 1.5, 0.0]))


def star(a: np.ndarray, phi: np.ndarray, name: str = "star") -> Curve:
    """Star curve r(theta) = 1 + sum_{k=2}^{8} a_k cos(k theta + phi_k).

    The polar form is rewritten exactly as a degree-9 trigonometric
    polynomial via product-to-sum identities.
    """
    ks = np.arange(2, 2 + len(a))
    D = int(ks[-1]) + 1
    cx = np.zeros(D + 1); sx = np.zeros(D + 1)
    cy = np.zeros(D + 1); sy = np.zeros(D + 1)
    cx[1] += 1.0
    sy[1] += 1.0
    for k, ak, ph in zip(ks, a, phi):
        c, s = np.cos(ph), np.sin(ph)
        # a cos(k t + ph) cos t = a/2 [cos((k+1)t + ph) + cos((k-1)t + ph)]
        # a cos(k t + ph) sin t = a/2 [sin((k+1)t + ph) - sin((k-1)t + ph)]
        for m, sgn in ((k + 1, 1.0), (k - 1, -1.0)):
            cx[m] += 0.5 * ak * c
            sx[m] -= 0.5 * ak * s
            cy[m] += sgn * 0.5 * ak * s
            sy[m] += sgn * 0.5 * ak * c
    return Curve(name, cx, sx, cy, sy)


def star_pool(n: int, seed: int = 0):
    """n star curves with a_k ~ U(0, 0.15/k), phi_k ~ U(0, 2 pi), k = 2..8."""
    rng = np.random.default_rng(seed)
    ks = np.arange(2, 9)
    out = []
    for i in range(n):
        a = rng.uniform(0.0, 0.15 / ks)
        phi = rng.uniform(0.0, 2.0 * np.pi, size=len(ks))
        out.append(star(a, phi, name=f"star{seed}_{i}"))
    return out


def curve_points(curve: Curve, s: np.ndarray) -> np.ndarray:
    """Points on the curve (for placing observation points); shape (len(s), 2)."""
    d = np.arange(curve.degree + 1)[:, None]
    c, sn = np.cos(d * s[None, :]), np.sin(d * s[None, :])
    return np.stack([curve.cx @ c + curve.sx @ sn, curve.cy @ c + curve.sy @ sn], axis=1)


# --------------------------------------------------------------------------
# Incident signals (uniform samples of f; u_inc = f(t - p.r/c))
# --------------------------------------------------------------------------
@dataclass
class Signal:
    t0: float
    dt: float
    f: np.ndarray          # samples f(t0 + n dt), n = 0..len(f)-1

    @property
    def t(self):
        return self.t0 + self.dt * np.arange(len(self.f))


def _smoothstep(x):
    """C-infinity step: 0 for x <= 0, 1 for x >= 1 (exp(-1/x) construction)."""
    x = np.asarray(x, dtype=float)
    out = np.zeros_like(x)
    inside = (x > 0) & (x < 1)
    xi = x[inside]
    ea = np.exp(-1.0 / xi)
    eb = np.exp(-1.0 / (1.0 - xi))
    out[inside] = ea / (ea + eb)
    out[x >= 1] = 1.0
    return out


def gaussian_pulse(t0=-1.0, t1=10.0, dt=1.0 / 256, center=4.0, var2=0.5, freq=6.0) -> Signal:
    """f(t) = exp(-(t - center)^2 / var2) cos(freq t), sampled on [t0, t1]."""
    n = int(round((t1 - t0) / dt)) + 1
    t = t0 + dt * np.arange(n)
    return Signal(t0, dt, np.exp(-(t - center) ** 2 / var2) * np.cos(freq * t))


def gaussian_pulse_value(t, center=4.0, var2=0.5, freq=6.0):
    """(f(t), f'(t)) of f(t) = exp(-(t - center)^2 / var2) cos(freq t), any real t."""
    t = np.asarray(t, dtype=float)
    e = np.exp(-(t - center) ** 2 / var2)
    return e * np.cos(freq * t), e * (-2.0 * (t - center) / var2 * np.cos(freq * t) - freq * np.sin(freq * t))


def plane_pulses_on_boundary(x, nu, waves, t0, dt, n_t, c=1.0):
    """Dirichlet data of a general incident field on a boundary: the sum of
    plane-wave pulses u_inc(r, t) = sum_w amp_w f_w(t - p_w.r / c - delay_w),
    f_w a gaussian_pulse_value with the wave's (center, var2, freq).  Given
    points x [N][2] and unit normals nu [N][2], returns the samples
    b = -u_inc(x_i, t_n) and db = -(nu_i . grad u_inc)(x_i, t_n) at t_n = t0 + n
    dt, n < n_t, both [n_t][N] (time-major).  waves: sequence of dicts with
    keys amp, p (unit 2-vector), delay, center, var2, freq."""
    x = np.asarray(x, dtype=float)
    nu = np.asarray(nu, dtype=float)
    t = t0 + dt * np.arange(n_t)
    b = np.zeros((n_t, len(x)))
    db = np.zeros((n_t, len(x)))
    for w in waves:
        p = np.asarray(w["p"], dtype=float)
        arg = t[:, None] - (x @ p)[None, :] / c - w["delay"]
        f, fp = gaussian_pulse_value(arg, w["center"], w["var2"], w["freq"])
        b -= w["amp"] * f
        db -= w["amp"] * fp * (-(nu @ p) / c)[None, :]
    return b, db


def two_pulse_field():
    """A general incident field for tests: two plane pulses from different
    directions with different carriers and delays (not one plane wave)."""
    return [dict(amp=1.0, p=(1.0, 0.0), delay=0.0, center=4.0, var2=0.5, freq=12.0),
            dict(amp=0.7, p=(-0.6, 0.8), delay=5.0, center=4.0, var2=0.3, freq=14.0)]


def general_pulses(n_waves: int = 24, t_span: float = 200.0, seed: int = 7):
    """A long general incident field: n_waves plane pulses with seeded unit
    directions, delays uniform in [0, t_span], carriers in [8, 30] and
    envelope widths var2 in [0.2, 1]; sampled on [-3, t_span + 14] (every
    pulse's envelope is below 1e-20 outside).  Returns dict(waves, t0, t1)."""
    rng = np.random.default_rng(seed)
    waves = []
    for _ in range(n_waves):
        a = rng.uniform(0.0, 2.0 * np.pi)
        waves.append(dict(amp=float(rng.uniform(0.5, 1.0)), p=(float(np.cos(a)), float(np.sin(a))),
                          delay=float(rng.uniform(0.0, t_span)), center=4.0, var2=float(rng.uniform(0.2, 1.0)),
                          freq=float(rng.uniform(8.0, 30.0))))
    return dict(waves=waves, t0=-3.0, t1=t_span + 14.0)


def chirp_value(t, t_end: float, rate: float = 4000.0, ramp: float = 5.0):
    """Chirp sin(g + g^2/rate), g = 4t + 6 cos(t / sqrt 12) (the paper's chirp
    incidence, Sec. 6.3, for rate = 4000), switched on over [0, ramp] and off
    over [t_end, t_end + ramp] with a C-infinity step so that the signal is
    compactly supported in [0, t_end + ramp].  Any real t."""
    t = np.asarray(t, dtype=float)
    T = t_end + ramp
    g = 4.0 * t + 6.0 * np.cos(t / np.sqrt(12.0))
    env = _smoothstep(t / ramp) * _smoothstep((T - t) / ramp)
    return env * np.sin(g + g * g / rate)


def chirp(t_end: float, dt: float, rate: float = 4000.0, ramp: float = 5.0) -> Signal:
    """chirp_value sampled at n dt, n = 0 .. ceil((t_end + ramp)/dt)."""
    n = int(np.ceil((t_end + ramp) / dt)) + 1
    t = dt * np.arange(n)
    return Signal(0.0, dt, chirp_value(t, t_end, rate, ramp))


# --------------------------------------------------------------------------
# Observation points and times
# --------------------------------------------------------------------------
def ring(n: int, radius: float, center=(0.0, 0.0)) -> np.ndarray:
    th = 2.0 * np.pi * np.arange(n) / n
    return np.stack([center[0] + radius * np.cos(th), center[1] + radius * np.sin(th)], axis=1)


# --------------------------------------------------------------------------
# Named workloads (plain parameter sets)
# --------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    curve: Curve
    W: float                      # band limit; frequencies omega_j = j W / F, j = 1..F
    F: int
    N: object                     # int (fixed N) or dict(ppw=, n_min=, n_mult=, n_cap=)
    direction: tuple = (1.0, 0.0)
    c: float = 1.0
    H: float = 10.0
    tau0: float = 0.0
    signal: Signal | None = None
    obs: np.ndarray | None = None
    times: np.ndarray | None = None
    extra: dict = field(default_factory=dict)


def circle_pulse() -> Workload:
    """Unit circle, N = 128, F = 64 on (0, 20], direction (1, 0), Gaussian
    pulse f = exp(-(t-4)^2/0.5) cos 6t, 16 observation points at radius 3,
    32 times on [0, 40]."""
    return Workload("circle_N128_F64", circle(1.0), 20.0, 64, 128,
                    H=4.0, tau0=3.0, signal=gaussian_pulse(),
                    obs=ring(16, 3.0), times=np.linspace(0.0, 40.0, 32))


def kite_chirp(F=512, W=200.0, n_obs=256, n_times=1024, t_far=1.0e4) -> Workload:
    """Kite, F frequencies on (0, W], 10 points per wavelength (multiple of 32,
    64 <= N <= 4096), chirp incidence to T = t_far, observation points on the
    circle of radius 3, half the times in [0, 100] and half in
    [t_far - 100, t_far]."""
    dt = np.pi / (4.0 * W)
    sig = chirp(t_far + 5.0, dt)
    half = n_times // 2
    times = np.concatenate([np.linspace(0.0, 100.0, half),
                            np.linspace(t_far - 100.0, t_far, n_times - half)])
    return Workload(f"kite_chirp_F{F}_W{int(W)}", kite(), W, F,
                    dict(ppw=10.0, n_min=64, n_mult=32, n_cap=4096),
                    direction=(1.0, 0.0), H=3.0, tau0=2.25, signal=sig,
                    obs=ring(n_obs, 3.0), times=times)


def kite_n1024(F=1024, n_obs=256, n_times=1024, t_far=1.0e4) -> Workload:
    """Solve-throughput workload: kite, N = 1024 at every frequency (10 points
    per wavelength at the top frequency 69), F = 1024 frequencies on (0, 69],
    one plane-wave direction (1, 0); a slow chirp (rate 16000, band below 40)
    to T = t_far observed on 256 points of the circle of radius 3 at 512 times
    in [0, 100] and 512 in [t_far - 100, t_far]."""
    W = 69.0
    dt = np.pi / (4.0 * W)
    sig = chirp(t_far + 5.0, dt, rate=16000.0)
    half = n_times // 2
    times = np.concatenate([np.linspace(0.0, 100.0, half),
                            np.linspace(t_far - 100.0, t_far, n_times - half)])
    return Workload(f"kite_N1024_F{F}", kite(), W, F, 1024, direction=(1.0, 0.0),
                    H=10.0, tau0=10.0, signal=sig, obs=ring(n_obs, 3.0), times=times)


def star_batch(n_curves=64, F=256, W=120.0, seed=0) -> dict:
    """The batching configuration: n_curves seeded star curves, each with F
    frequencies on (0, W] and N from 17 points per wavelength (multiple of 32,
    64 <= N <= 2048), FP64, one plane-wave direction (1, 0)."""
    return dict(curves=star_pool(n_curves, seed), W=W, F=F,
                rule=dict(ppw=17.0, n_min=64, n_mult=32, n_cap=2048), direction=(1.0, 0.0))


def interior_points(curve: Curve, n: int, seed: int = 3, shrink: float = 0.5) -> np.ndarray:
    """Points well inside a star-shaped-about-its-centroid curve (used for the
    interior-extinction checks): shrink curve points toward the centroid."""
    rng = np.random.default_rng(seed)
    s = rng.uniform(0, 2 * np.pi, n)
    pts = curve_points(curve, s)
    cen = curve_points(curve, np.linspace(0, 2 * np.pi, 256, endpoint=False)).mean(axis=0)
    lam = rng.uniform(0.0, shrink, n)[:, None]
    return cen + lam * (pts - cen)


def serve_requests(rate: float, duration: float, seed: int = 1, pool: int = 16, dw: float = 1.0):
    """The serving configuration: Poisson arrivals at `rate` per second over
    `duration` seconds.  Each request names a star curve of a seeded pool (the
    batching configuration's curves), a band [lo, lo + B] with B ~ U(10, 50)
    and lo ~ U(0, 300 - B) snapped to the grid dw (so j_first = floor(lo/dw)
    and F = round(B/dw) frequencies (j_first + j) dw, j = 1..F), one N ~
    U{256, 288, ..., 4096} and 1..64 plane waves at uniform angles.
    Returns (curves, requests): requests in arrival order, dicts with
    t, curve, j_first, F, N, dirs ([n_rhs][2])."""
    rng = np.random.default_rng(seed)
    curves = star_pool(pool, 0)
    reqs = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t > duration:
            break
        B = rng.uniform(10.0, 50.0)
        lo = rng.uniform(0.0, 300.0 - B)
        N = 256 + 32 * int(rng.integers(0, 121))
        n_rhs = int(rng.integers(1, 65))
        ang = rng.uniform(0.0, 2.0 * np.pi, n_rhs)
        reqs.append(dict(t=t, curve=int(rng.integers(0, pool)), j_first=int(np.floor(lo / dw)),
                         F=max(1, int(round(B / dw))), N=N, dirs=np.stack([np.cos(ang), np.sin(ang)], axis=1)))
    return curves, reqs
