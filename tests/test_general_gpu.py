"""General incident fields (Sec. 3.2, eq. bkdef2) on the GPU, through the C
ABI: sampled Dirichlet data -u_inc at the nodes, windowed node by node, each
window's exterior Dirichlet problem by the combined potential on a plan of
that formulation (fhw_solve_general), each window's field
(fhw_eval_field_windows) and the per-window synthesis (fhw_synthesize_windows),
against the oracle's boundary_window_transforms / assemble_dirichlet /
field_dirichlet / synthesize_windowed on the same seeded field (two plane
pulses from different directions: not one plane wave).  Each side computes
its own nodes and samples the field there.

  * small sizes, both precisions, kite and circle: densities of every window
    and frequency, fields and time samples, element by element;
  * ragged shapes: N = 300 (two 256-node tiles, the second ragged) and F =
    100 frequencies (not a multiple of the kernel's 8-system groups);
  * a subset of windows equals the matching blocks of the whole set;
  * full size (kite, N = 1024, F = 1024, W = 69): sampled frequencies of every
    window against the oracle;
  * the low-frequency decomposition for general data (the circle
    configuration): against the oracle's whole path and the exact
    time-domain solution;
  * argument and state errors."""
import numpy as np
import pytest
import torch

import oracle as O
import workloads as Wk

pytestmark = pytest.mark.gpu


def say(*a):
    print("CASE", *a, flush=True)


def relmax(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def fhw():
    from paper_1807_02718_amd import fhw as m
    return m


FIELD = Wk.two_pulse_field()
T0, T1 = -3.0, 18.0


def gpu_boundary(ctx, N, dt):
    """Samples of the field at the library's own nodes, time-major, on the device."""
    g = ctx.geometry(N).cpu().numpy()
    x, nu = g[0:2].T, g[7:9].T
    n_t = int(round((T1 - T0) / dt)) + 1
    b, _ = Wk.plane_pulses_on_boundary(x, nu, FIELD, T0, dt, n_t)
    return torch.as_tensor(b, device="cuda")


def oracle_boundary(curve, N, dt):
    gm = O.geometry(curve, N)
    n_t = int(round((T1 - T0) / dt)) + 1
    b, _ = Wk.plane_pulses_on_boundary(gm["x"], gm["nu"], FIELD, T0, dt, n_t)
    return gm, b.T        # the oracle takes [N][n_t]


def oracle_densities(curve, N, W, F, H, dt, ks, js):
    """phi[q][jj] for windows ks and frequency indices js (omega = (j+1) W/F)."""
    gm, b = oracle_boundary(curve, N, dt)
    omega, kappa = O.frequency_grid(W, F)
    eta = O.coupling(kappa)
    Bk = O.boundary_window_transforms(b, T0, dt, H, ks, omega[js])
    out = np.zeros((len(ks), len(js), N), dtype=complex)
    for jj, j in enumerate(js):
        A = O.assemble_dirichlet(gm, kappa[j], eta[j])
        for q in range(len(ks)):
            out[q, jj] = np.linalg.solve(A, Bk[q, jj])
    return gm, out


def oracle_field(gm, phi, j, W, F, obs):
    omega, kappa = O.frequency_grid(W, F)
    eta = O.coupling(kappa)
    return O.field_dirichlet(gm, phi, kappa[j], eta[j], obs)


CASES = [("kite", Wk.kite(), 96, "fp64"), ("kite", Wk.kite(), 96, "fp32_refine"), ("circle", Wk.circle(1.0), 64, "fp64")]


@pytest.mark.parametrize("name,curve,N,precision", CASES, ids=[f"{c[0]}-{c[3]}" for c in CASES])
def test_general_path_matches_oracle(fhw, name, curve, N, precision):
    W, F, H, tau0, dt = 20.0, 128, 4.0, 3.0, 1.0 / 128
    obs = Wk.ring(8, 3.0)
    times = np.linspace(-2.0, 70.0, 90)
    b_o = oracle_boundary(curve, N, dt)[1]
    u_ref, ks = O.run_general(curve, W, F, N, b_o, T0, dt, H, tau0, obs, times)
    ctx = fhw.Context()
    try:
        say("general path", name, "N", N, "F", F, precision, "windows", list(ks))
        ctx.plan(curve, W, F, N=N, precision=precision, refine_tol=1e-13, refine_max=10, formulation="combined")
        ctx.factor()
        b = gpu_boundary(ctx, N, dt)
        psi, res, sw, k_first = ctx.solve_general(b, T0, dt, H)
        assert k_first == ks[0] and psi.shape[0] == len(ks)
        V = ctx.eval_field_windows(psi, obs)
        u = ctx.synthesize_windows(H, tau0, k_first, V, times).cpu().numpy()
        psi_h, V_h = psi.cpu().numpy(), V.cpu().numpy()
    finally:
        ctx.close()
    js = np.arange(F)
    gm, ref_psi = oracle_densities(curve, N, W, F, H, dt, ks, js)
    e_psi = max(relmax(psi_h[q].reshape(F, N), ref_psi[q]) for q in range(len(ks)))
    omega, kappa = O.frequency_grid(W, F)
    Vref = np.stack([O.field_full_grid(np.stack([oracle_field(gm, ref_psi[q, j], j, W, F, obs) for j in js], axis=1),
                                       0.0) for q in range(len(ks))])
    e_V = relmax(V_h, Vref)
    e_u = relmax(u, u_ref)
    say("general path", name, precision, "psi", e_psi, "V", e_V, "u", e_u, "max |u|", float(np.abs(u_ref).max()))
    bar = 1e-11 if precision == "fp64" else 1e-10
    assert e_psi < bar and e_V < bar and e_u < 1e-10
    if precision == "fp32_refine":
        assert np.all(res <= 1e-13) and np.all(sw >= 1)


def test_general_ragged_shapes(fhw):
    """N = 300 nodes (a full and a ragged 256-node tile of the right-hand-side
    kernel) and F = 100 systems (groups of 8 with a ragged last group):
    densities and fields against the oracle on sampled frequencies."""
    curve, N, W, F, H, dt = Wk.kite(), 300, 30.0, 100, 3.0, 1.0 / 100
    obs = Wk.ring(5, 2.5)
    ctx = fhw.Context()
    try:
        say("general ragged: N", N, "F", F)
        ctx.plan(curve, W, F, N=N, precision="fp64", formulation="combined")
        ctx.factor()
        b = gpu_boundary(ctx, N, dt)
        psi, _, _, k_first = ctx.solve_general(b, T0, dt, H)
        V = ctx.eval_field_windows(psi, obs).cpu().numpy()
        psi_h = psi.cpu().numpy()
    finally:
        ctx.close()
    ks = O.window_indices(T0, T1, H)
    assert k_first == ks[0] and psi_h.shape[0] == len(ks)
    js = np.array([0, 7, 8, 50, 96, 99])
    gm, ref = oracle_densities(curve, N, W, F, H, dt, ks, js)
    omega, kappa = O.frequency_grid(W, F)
    for q in range(len(ks)):
        got = psi_h[q].reshape(F, N)[js]
        e = relmax(got, ref[q])
        Vq = np.stack([oracle_field(gm, ref[q, jj], j, W, F, obs) for jj, j in enumerate(js)], axis=1)
        eV = relmax(V[q][:, F + 1 + js[js < F - 1]], Vq[:, js < F - 1])
        say("window", ks[q], "psi", e, "V", eV)
        assert e < 1e-11 and eV < 1e-11


def test_general_window_subset(fhw):
    """Windows k_first + 1 .. k_first + 2 alone give the matching blocks of
    the solve over every window (same kernels, other group positions)."""
    curve, N, W, F, H, dt = Wk.kite(), 64, 20.0, 64, 4.0, 1.0 / 64
    ctx = fhw.Context()
    try:
        say("general window subset")
        ctx.plan(curve, W, F, N=N, precision="fp64", formulation="combined")
        ctx.factor()
        b = gpu_boundary(ctx, N, dt)
        full, _, _, k0 = ctx.solve_general(b, T0, dt, H)
        part, _, _, _ = ctx.solve_general(b, T0, dt, H, k_first=k0 + 1, n_win=2)
        full_h, part_h = full.cpu().numpy(), part.cpu().numpy()
    finally:
        ctx.close()
    assert relmax(part_h, full_h[1:3]) < 1e-14


def test_general_full_size_sampled(fhw):
    """Kite at N = 1024, F = 1024 on (0, 69] (the solve-throughput workload's
    systems) with the two-pulse field, H = 10: every window's densities at
    sampled frequencies and its field at sampled points against the oracle.
    The error is taken relative to the largest sampled value: far from the
    carriers a transform is a sum of ~1800 terms that cancels to between 1e-5
    (omega near 0) and 1e-10 (omega near W) of the sum of their magnitudes,
    so its own relative error is the summation order's rounding over that."""
    wl = Wk.kite_n1024()
    N, W, F, H = 1024, wl.W, wl.F, 10.0
    dt = np.pi / (4.0 * W)
    obs = Wk.ring(4, 3.0)
    for precision in ("fp64", "fp32_refine"):
        ctx = fhw.Context()
        try:
            say("general full size", precision)
            ctx.plan(wl.curve, W, F, N=N, precision=precision, refine_tol=1e-12, refine_max=10,
                     formulation="combined")
            ctx.factor()
            b = gpu_boundary(ctx, N, dt)
            psi, res, _, k_first = ctx.solve_general(b, T0, dt, H)
            V = ctx.eval_field_windows(psi, obs).cpu().numpy()
            psi_h = psi.cpu().numpy()
            del b, psi
        finally:
            ctx.close()
        ks = O.window_indices(T0, T1, H)
        assert k_first == ks[0] and psi_h.shape[0] == len(ks)
        # the lowest and highest frequencies, and two at the pulses' carriers
        # (12 and 14), which set the scale of the relative error
        js = np.array([0, 177, 206, 511, 1022])
        gm, ref = oracle_densities(wl.curve, N, W, F, H, dt, ks, js)
        omega, kappa = O.frequency_grid(W, F)
        for q in range(len(ks)):
            e = relmax(psi_h[q].reshape(F, N)[js], ref[q])
            Vq = np.stack([oracle_field(gm, ref[q, jj], j, W, F, obs) for jj, j in enumerate(js)], axis=1)
            eV = relmax(V[q][:, F + 1 + js], Vq)
            say("full size", precision, "window", ks[q], "psi", e, "V", eV)
            assert e < 1e-10 and eV < 1e-10
        if precision == "fp32_refine":
            assert np.all(res <= 1e-12)


def test_general_errors(fhw):
    say("general argument and state errors")
    ctx = fhw.Context()
    try:
        ctx.plan(Wk.kite(), 20.0, 64, N=64)          # the direct formulation
        b = gpu_boundary(ctx, 64, 1.0 / 64)
        ctx.factor()
        with pytest.raises(fhw.FhwError) as e:
            ctx.solve_general(b, T0, 1.0 / 64, 4.0)
        assert e.value.code == fhw.FHW_E_STATE
        ctx.plan(Wk.kite(), 20.0, 64, N=64, formulation="combined")
        with pytest.raises(fhw.FhwError) as e:          # no resident factors yet
            ctx.solve_general(b, T0, 1.0 / 64, 4.0)
        assert e.value.code == fhw.FHW_E_STATE
        ctx.factor()
        for call in (lambda: ctx.solve_densities(), lambda: ctx.solve_incidences([("plane", (1.0, 0.0))]),
                     lambda: ctx.eval_field(torch.zeros(int(ctx.psi_off[-1]), dtype=torch.complex128, device="cuda"),
                                            Wk.ring(2, 3.0))):
            with pytest.raises(fhw.FhwError) as e:      # direct calls on a combined plan
                call()
            assert e.value.code == fhw.FHW_E_STATE
        with pytest.raises(fhw.FhwError) as e:          # samples at another N
            ctx.solve_general(b[:, :32].contiguous(), T0, 1.0 / 64, 4.0)
        assert e.value.code == fhw.FHW_E_INVALID
        with pytest.raises(fhw.FhwError) as e:          # no windows
            ctx.solve_general(b, T0, 1.0 / 64, 4.0, k_first=1, n_win=0)
        assert e.value.code == fhw.FHW_E_INVALID
        with pytest.raises(fhw.FhwError) as e:
            ctx.solve_general(b, T0, 0.0, 4.0, k_first=1, n_win=2)
        assert e.value.code == fhw.FHW_E_INVALID
        psi, _, _, k0 = ctx.solve_general(b, T0, 1.0 / 64, 4.0)
        with pytest.raises(fhw.FhwError) as e:          # no graded nodes in this plan
            ctx.eval_field_windows_lowfreq(psi, Wk.ring(2, 3.0),
                                           V_sing=torch.empty((psi.shape[0], 2, 129), dtype=torch.complex128,
                                                              device="cuda"))
        assert e.value.code == fhw.FHW_E_STATE
        with pytest.raises(fhw.FhwError) as e:          # the combined formulation needs a fixed N
            ctx.plan(Wk.kite(), 20.0, 64, ppw=8.0, n_min=32, n_mult=16, n_cap=256, formulation="combined")
        assert e.value.code == fhw.FHW_E_INVALID
    finally:
        ctx.close()
    with pytest.raises(fhw.FhwError):
        fhw.window_range(1.0, 0.0, 4.0)


def _circle_V(kappa, robs, thobs):
    """Exact scattered-field series of the unit circle, p = (1, 0)."""
    from scipy import special
    if kappa == 0.0:
        return np.ones(len(robs), dtype=complex)
    mmax = int(1.3 * kappa * max(1.0, np.max(robs))) + (40 if kappa > 1 else 12)
    ms = np.arange(-mmax, mmax + 1)
    return ((1j ** ms) * special.jv(ms, kappa) * special.hankel1(ms, kappa * robs[:, None]) / special.hankel1(ms, kappa)
            * np.exp(1j * np.outer(thobs, ms))).sum(1)


def _exact_trace(robs, thobs, times):
    """(1/pi) Re int_0^inf A V e^{-i w t} dw for the pulse a = -e^{-(t-4)^2/0.5}
    cos 6t, by Gauss-Legendre on a mesh graded toward w = 0."""
    w_ = lambda w: -0.5 * sum(np.sqrt(np.pi * 0.5) * np.exp(4j * (w + sg * 6.0)) * np.exp(-0.5 * (w + sg * 6.0) ** 2 / 4)
                              for sg in (1.0, -1.0))
    edges = [0.0] + [2.0 ** -k for k in range(60, 0, -1)] + list(np.arange(1.0, 30.0001, 0.25))
    x, wg = np.polynomial.legendre.leggauss(40)
    ws = np.concatenate([0.5 * (a + b) + 0.5 * (b - a) * x for a, b in zip(edges[:-1], edges[1:])])
    ww = np.concatenate([0.5 * (b - a) * wg for a, b in zip(edges[:-1], edges[1:])])
    V = np.stack([_circle_V(w, robs, thobs) for w in ws], axis=1)
    return ((w_(ws)[None, :] * V * ww[None, :]) @ np.exp(-1j * np.outer(ws, times))).real / np.pi


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_general_lowfreq_circle(fhw, precision):
    """The circle configuration (W = 20, F = 256, omega_c = 1.25, M = 16, n =
    8, q = 9.1, N = 128, H = 4, tau0 = 3) with the pulse given as general
    Dirichlet data: solves at the grid and graded frequencies, both window
    fields, fhw_synthesize_windows_lowfreq; against the oracle's whole path
    (run_general with the decomposition) and the exact time-domain solution."""
    sig = Wk.gaussian_pulse()
    W, F, N, H, tau0 = 20.0, 256, 128, 4.0, 3.0
    LF = dict(jc=16, M=16, n=8, q=9.1)
    obs = Wk.ring(16, 3.0)[::4]
    times = np.linspace(0.0, 40.0, 32)
    wave = dict(amp=1.0, p=(1.0, 0.0), delay=0.0, center=4.0, var2=0.5, freq=6.0)
    gm = O.geometry(Wk.circle(1.0), N)
    b_o, _ = Wk.plane_pulses_on_boundary(gm["x"], gm["nu"], [wave], sig.t0, sig.dt, len(sig.f))
    u_ref, ks = O.run_general(Wk.circle(1.0), W, F, N, b_o.T, sig.t0, sig.dt, H, tau0, obs, times, lowfreq=LF)
    ex = _exact_trace(np.hypot(obs[:, 0], obs[:, 1]), np.arctan2(obs[:, 1], obs[:, 0]), times)
    ctx = fhw.Context()
    try:
        say("general lowfreq circle", precision)
        ctx.plan(Wk.circle(1.0), W, F, N=N, precision=precision, refine_tol=1e-13, refine_max=10, lowfreq=LF,
                 formulation="combined")
        ctx.factor()
        g = ctx.geometry(N).cpu().numpy()
        b, _ = Wk.plane_pulses_on_boundary(g[0:2].T, g[7:9].T, [wave], sig.t0, sig.dt, len(sig.f))
        psi, res, _, k_first = ctx.solve_general(torch.as_tensor(b, device="cuda"), sig.t0, sig.dt, H)
        assert k_first == ks[0] and psi.shape[0] == len(ks)
        V = ctx.eval_field_windows(psi, obs)
        Vs = ctx.eval_field_windows_lowfreq(psi, obs)
        u = ctx.synthesize_windows_lowfreq(H, tau0, k_first, V, Vs, times).cpu().numpy()
    finally:
        ctx.close()
    e_o, e_x = relmax(u, u_ref), relmax(u, ex)
    say("general lowfreq circle", precision, "vs oracle", e_o, "vs exact", e_x, "oracle vs exact", relmax(u_ref, ex))
    assert e_o < 1e-10 and e_x < 1e-9
