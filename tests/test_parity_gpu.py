"""GPU-vs-oracle parity for every step of the hot path, through the C ABI.

Tolerances (relative, max norm): matrices 1e-13 (normwise per frequency),
FP64 densities 1e-11, fields 1e-11, time samples 1e-10; Bessel values a few
ulps plus the argument's conditioning.  Each test prints the case it runs.
"""
import numpy as np
import pytest
import torch
from scipy import special

import oracle as O
import workloads as Wk

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fhw():
    from paper_1807_02718_amd import fhw as m
    return m


@pytest.fixture
def ctx(fhw):
    c = fhw.Context()
    yield c
    c.close()


def say(*a):
    print("CASE", *a, flush=True)


def relmax(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


# ---------------------------------------------------------------- Bessel (a3)
def test_hankel01_values(ctx):
    say("hankel01")
    brk = np.array([3.0, 4.5, 6.75, 10.0, 15.0, 25.0])
    z = np.concatenate([np.geomspace(1e-5, 1e5, 4000), brk, np.nextafter(brk, 0), np.nextafter(brk, 10)])
    h = ctx.hankel01(z).cpu().numpy()
    eps = np.finfo(float).eps
    cond = 8 * eps * np.sqrt(np.maximum(z, 1.0))
    for col, (fj, fy) in enumerate(((special.j0, special.y0), (special.j1, special.y1))):
        J, Y = fj(z), fy(z)
        errJ = np.abs(h[:, col].real - J) - cond
        errY = np.abs(h[:, col].imag - Y) - cond
        assert np.max(errJ / np.maximum(1.0, np.abs(J))) < 6e-15
        assert np.max(errY / np.maximum(1.0, np.abs(Y))) < 6e-15


# ------------------------------------------------------- geometry, Kress (a1, a2)
@pytest.mark.parametrize("curve,N", [(Wk.circle(1.0), 64), (Wk.kite(), 256), (Wk.star_pool(1, 0)[0], 96)])
def test_geometry_and_kress(ctx, curve, N):
    say("geometry", curve.name, N)
    ctx.plan(curve, 10.0, 4, N=N)
    g = ctx.geometry(N).cpu().numpy()
    ref = O.geometry(curve, N)
    assert np.max(np.abs(g[0:2].T - ref["x"])) < 1e-14
    assert np.max(np.abs(g[2:4].T - ref["dx"])) < 1e-13
    assert np.max(np.abs(g[4:6].T - ref["ddx"])) < 1e-12
    assert np.max(np.abs(g[6] - ref["speed"])) < 1e-13
    assert np.max(np.abs(g[7:9].T - ref["nu"])) < 1e-14
    R, L = ctx.kress_weights(N)
    assert np.max(np.abs(R.cpu().numpy() - O.kress_weights(N))) < 1e-14
    assert np.max(np.abs(L.cpu().numpy()[1:] - O.kress_log_table(N)[1:])) < 1e-13


# ------------------------------------------------------------- assembly (a3)
@pytest.mark.parametrize("curve,W,F,N", [(Wk.circle(1.0), 20.0, 8, 128), (Wk.kite(), 40.0, 6, 256),
                                          (Wk.star_pool(2, 0)[1], 30.0, 4, 160)])
def test_assembly(ctx, curve, W, F, N):
    say("assembly", curve.name, W, F, N)
    ctx.plan(curve, W, F, N=N, direction=(0.6, 0.8))
    mats, vecs = ctx.assemble(0, F)
    omega, kappa = O.frequency_grid(W, F)
    eta = O.coupling(kappa)
    gm = O.geometry(curve, N)
    for j in range(F):
        A = O.assemble(gm, kappa[j], eta[j])
        g = O.rhs_plane_wave(gm, kappa[j], eta[j], (0.6, 0.8))
        assert relmax(mats[j].cpu().numpy(), A) < 1e-13, j
        assert relmax(vecs[j].cpu().numpy(), g) < 1e-13, j


def test_assembly_ragged(ctx):
    say("assembly ragged kite")
    Ns, off = ctx.plan(Wk.kite(), 60.0, 12, ppw=6.0, n_min=32, n_mult=32, n_cap=4096)
    omega, kappa = O.frequency_grid(60.0, 12)
    Nref = O.discretization_sizes(kappa, O.curve_length(Wk.kite()), 6.0, 32, 32, 4096)
    assert np.array_equal(Ns, Nref)
    mats, vecs = ctx.assemble(3, 9)
    eta = O.coupling(kappa)
    for q in range(9):
        j = 3 + q
        gm = O.geometry(Wk.kite(), int(Ns[j]))
        assert relmax(mats[q].cpu().numpy(), O.assemble(gm, kappa[j], eta[j])) < 1e-13


# ------------------------------------------------------------------- LU (a4, a5)
def _rand_batch(Ns, seed, dtype=torch.complex128):
    rng = np.random.default_rng(seed)
    mats = [rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) for n in Ns]
    rhs = [rng.standard_normal(n) + 1j * rng.standard_normal(n) for n in Ns]
    flat = torch.tensor(np.concatenate([m.ravel(order="F") for m in mats]), dtype=dtype, device="cuda")
    b = torch.tensor(np.concatenate(rhs), dtype=torch.complex128, device="cuda")
    return mats, rhs, flat, b


@pytest.mark.parametrize("Ns", [[1, 2, 3, 17, 63, 64, 65, 100, 128, 200, 257], [1100], [2100, 130], [4096]])
def test_lu_random_fp64(ctx, Ns):
    say("lu fp64", Ns)
    mats, rhs, flat, b = _rand_batch(Ns, seed=len(Ns) + Ns[0])
    fac = ctx.lu_factor(flat, Ns)
    x = ctx.lu_solve(fac, b).cpu().numpy()
    o = 0
    for A, g, n in zip(mats, rhs, Ns):
        ref, _ = O.solve_density(A, g)
        xs = x[o:o + n]
        o += n
        cond = np.linalg.cond(A)
        assert relmax(xs, ref) < 1e-15 * cond * n + 1e-13, (n, cond)
        # normwise backward error, against LAPACK's on the same system
        nA = np.linalg.norm(A)
        be = np.linalg.norm(A @ xs - g) / (nA * np.linalg.norm(xs))
        be_ref = np.linalg.norm(A @ ref - g) / (nA * np.linalg.norm(ref))
        assert be < 10 * be_ref + 1e-16, (n, be, be_ref)


def test_lu_pivots_match_lapack(ctx):
    say("lu pivots")
    from scipy import linalg
    Ns = [5, 64, 130]
    mats, rhs, flat, b = _rand_batch(Ns, seed=11)
    fac = ctx.lu_factor(flat, Ns)
    piv = fac["piv"].cpu().numpy()
    o = 0
    for A, n in zip(mats, Ns):
        _, p_ref = linalg.lu_factor(A)
        assert np.array_equal(piv[o:o + n], p_ref), n
        o += n


def test_lu_random_fp32(ctx):
    say("lu fp32")
    Ns = [16, 64, 200, 300]
    mats, rhs, flat, b = _rand_batch(Ns, seed=5, dtype=torch.complex64)
    fac = ctx.lu_factor(flat, Ns, precision="fp32_refine")
    x = ctx.lu_solve(fac, b).cpu().numpy()
    o = 0
    for A, g, n in zip(mats, rhs, Ns):
        ref = np.linalg.solve(A.astype(np.complex64).astype(np.complex128), g)
        xs = x[o:o + n]
        o += n
        assert relmax(xs, ref) < 3e-7 * np.linalg.cond(A), n


def test_lu_random_wide_batch_pivoting(ctx):
    """More than 256 matrices (the 256-thread panels and solves of large
    batches), random and so pivoting in most columns, ragged orders across
    several panels: the solves' pivot replays run with real exchanges (the
    BIE systems of the other large-batch tests rarely exchange rows).  FP64
    against LAPACK with its pivots, FP32 factors against the FP32-rounded
    matrices."""
    from scipy import linalg
    rng = np.random.default_rng(23)
    Ns = [int(n) for n in rng.integers(60, 200, size=300)]
    say("lu wide batch pivoting", len(Ns), min(Ns), max(Ns))
    mats, rhs, flat, b = _rand_batch(Ns, seed=29)
    fac = ctx.lu_factor(flat, Ns)
    x = ctx.lu_solve(fac, b).cpu().numpy()
    piv = fac["piv"].cpu().numpy()
    o = 0
    moved = 0
    for q, (A, g, n) in enumerate(zip(mats, rhs, Ns)):
        xs = x[o:o + n]
        ref, _ = O.solve_density(A, g)
        assert relmax(xs, ref) < 1e-15 * np.linalg.cond(A) * n + 1e-13, (q, n)
        if q % 25 == 0:
            _, p_ref = linalg.lu_factor(A)
            assert np.array_equal(piv[o:o + n], p_ref), (q, n)
        moved += int(np.count_nonzero(piv[o:o + n] != np.arange(n)))
        o += n
    assert moved > sum(Ns) // 2   # the replays really exchange rows
    mats32, rhs32, flat32, b32 = _rand_batch(Ns, seed=31, dtype=torch.complex64)
    fac32 = ctx.lu_factor(flat32, Ns, precision="fp32_refine")
    x32 = ctx.lu_solve(fac32, b32).cpu().numpy()
    o = 0
    for q, (A, g, n) in enumerate(zip(mats32, rhs32, Ns)):
        ref = np.linalg.solve(A.astype(np.complex64).astype(np.complex128), g)
        assert relmax(x32[o:o + n], ref) < 3e-7 * np.linalg.cond(A), (q, n)
        o += n


def test_lu_singular_reports(ctx, fhw):
    say("lu singular")
    flat = torch.zeros(64 * 64, dtype=torch.complex128, device="cuda")
    with pytest.raises(fhw.FhwError) as e:
        ctx.lu_factor(flat, [64])
    assert e.value.code == fhw.FHW_E_SINGULAR


# ---------------------------------------------------------- densities (a3-a5)
@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_densities_circle(ctx, precision):
    say("densities circle", precision)
    wl = Wk.circle_pulse()
    ctx.plan(wl.curve, wl.W, wl.F, N=wl.N, precision=precision, refine_tol=1e-14, refine_max=8)
    psi, res, sw = ctx.solve_densities(compute_resid=True)
    psi = psi.cpu().numpy()
    omega, kappa = O.frequency_grid(wl.W, wl.F)
    eta = O.coupling(kappa)
    gm = O.geometry(wl.curve, wl.N)
    for j in range(wl.F):
        ref, _ = O.solve_density(O.assemble(gm, kappa[j], eta[j]), O.rhs_plane_wave(gm, kappa[j], eta[j], (1.0, 0.0)))
        assert relmax(psi[j * wl.N:(j + 1) * wl.N], ref) < 1e-11, j
    assert np.all(res < 1e-13)


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_densities_kite_ragged(ctx, precision):
    say("densities kite ragged", precision)
    W, F = 30.0, 16
    Ns, off = ctx.plan(Wk.kite(), W, F, ppw=10.0, n_min=64, n_mult=32, n_cap=4096, precision=precision,
                       refine_tol=1e-14, refine_max=8, direction=(0.6, 0.8))
    psi, res, sw = ctx.solve_densities(compute_resid=True)
    psi = psi.cpu().numpy()
    omega, kappa = O.frequency_grid(W, F)
    eta = O.coupling(kappa)
    for j in range(F):
        gm = O.geometry(Wk.kite(), int(Ns[j]))
        ref, _ = O.solve_density(O.assemble(gm, kappa[j], eta[j]), O.rhs_plane_wave(gm, kappa[j], eta[j], (0.6, 0.8)))
        assert relmax(psi[off[j]:off[j + 1]], ref) < 1e-11, (j, Ns[j])


def test_densities_deterministic(ctx):
    say("determinism")
    ctx.plan(Wk.kite(), 20.0, 8, N=256)
    a = ctx.solve_densities()[0].clone()
    b = ctx.solve_densities()[0]
    assert torch.equal(a, b)


def test_refinement_noconv(ctx, fhw):
    say("refine noconv")
    ctx.plan(Wk.circle(1.0), 10.0, 2, N=64, precision="fp32_refine", refine_tol=1e-30, refine_max=0)
    with pytest.raises(fhw.FhwError) as e:
        ctx.solve_densities()
    assert e.value.code == fhw.FHW_E_NOCONV


def test_plan_rejects_bad_curves(ctx, fhw):
    say("plan errors")
    c = Wk.circle(1.0)
    cw = Wk.Curve("cw", c.cx, c.sx, c.cy, -c.sy)
    with pytest.raises(fhw.FhwError) as e:
        ctx.plan(cw, 10.0, 4, N=64)
    assert e.value.code == fhw.FHW_E_INVALID
    with pytest.raises(fhw.FhwError):
        ctx.plan(c, 10.0, 4, N=63)


# ------------------------------------------------------------------ field (a6)
def test_field(ctx, fhw):
    say("field")
    W, F = 24.0, 16
    ctx.plan(Wk.kite(), W, F, N=256, direction=(0.6, 0.8))
    psi, _, _ = ctx.solve_densities()
    obs = np.concatenate([Wk.ring(12, 3.0), [[2.0, 2.0], [-0.3, 0.2]]])
    V = ctx.eval_field(psi, obs, zero_value=1.0).cpu().numpy()
    omega, kappa = O.frequency_grid(W, F)
    eta = O.coupling(kappa)
    gm = O.geometry(Wk.kite(), 256)
    Vpos = np.zeros((len(obs), F), dtype=complex)
    for j in range(F):
        ref, _ = O.solve_density(O.assemble(gm, kappa[j], eta[j]), O.rhs_plane_wave(gm, kappa[j], eta[j], (0.6, 0.8)))
        Vpos[:, j] = O.field(gm, ref, kappa[j], obs)
    assert relmax(V, O.field_full_grid(Vpos, 1.0)) < 1e-11
    with pytest.raises(fhw.FhwError):
        ctx.eval_field(psi, np.array([[np.nan, 0.0]]))


# ------------------------------------------------------- synthesis (a7-a9)
def test_window_spectra(ctx):
    say("window spectra")
    sig = Wk.gaussian_pulse(t0=-1.0, t1=30.0, dt=1 / 128, center=12.0, var2=3.0, freq=5.0)
    W, F, H = 16.0, 64, 4.0
    ctx.plan(Wk.circle(1.0), W, F, N=32)
    ks = O.window_indices(sig.t[0], sig.t[-1], H)
    B = ctx.window_spectra(sig.f, sig.t0, sig.dt, H, int(ks[0]), len(ks)).cpu().numpy()
    wl = -W + (W / F) * np.arange(2 * F)
    ref = O.window_spectra(sig, H, ks, wl)
    assert relmax(B, ref) < 1e-12


def test_fourier_coefficients(ctx):
    say("fourier coefficients")
    W, F = 12.0, 128
    ctx.plan(Wk.circle(1.0), W, F, N=32)
    rng = np.random.default_rng(3)
    B = rng.standard_normal((3, 2 * F)) + 1j * rng.standard_normal((3, 2 * F))
    V = rng.standard_normal((5, 2 * F)) + 1j * rng.standard_normal((5, 2 * F))
    tau0 = 1.7
    c = ctx.fourier_coefficients(torch.tensor(B, device="cuda"), torch.tensor(V, device="cuda"), tau0).cpu().numpy()
    wl = -W + (W / F) * np.arange(2 * F)
    shift = np.exp(-1j * wl * tau0)
    for q in range(3):
        ref = O.fourier_coefficients(B[q][None, :] * V * shift[None, :], W)
        assert relmax(c[q], ref) < 1e-13


def test_fourier_coefficients_largest(ctx):
    """2F = 8192, the largest transform: a 128 KiB LDS buffer beside the
    static tables (one window, two points; the oracle's direct DFT)."""
    say("fourier coefficients, 2F = 8192")
    W, F = 40.0, 4096
    ctx.plan(Wk.circle(1.0), W, F, N=32)
    rng = np.random.default_rng(8)
    B = rng.standard_normal((1, 2 * F)) + 1j * rng.standard_normal((1, 2 * F))
    V = rng.standard_normal((2, 2 * F)) + 1j * rng.standard_normal((2, 2 * F))
    tau0 = 0.7
    c = ctx.fourier_coefficients(torch.tensor(B, device="cuda"), torch.tensor(V, device="cuda"), tau0).cpu().numpy()
    wl = -W + (W / F) * np.arange(2 * F)
    G = B[0][None, :] * V * np.exp(-1j * wl * tau0)[None, :]
    ref = O.fourier_coefficients(G, W)
    # the oracle's direct DFT evaluates exp at phases up to pi F: each term
    # carries a phase rounding of about eps pi F (2.9e-12 here), the FFT's
    # twiddles about one ulp
    err = relmax(c[0], ref)
    say("vs oracle", err)
    assert err < 8 * np.finfo(float).eps * np.pi * F
    # the same coefficients by the FFT identity pinned against the oracle on
    # the CPU: c_m = (-1)^m FFT(G)[m mod 2F] / 2F
    m = np.arange(-F, F)
    fft_ref = ((-1.0) ** m)[None, :] * np.fft.fft(G, axis=1)[:, m % (2 * F)] / (2 * F)
    assert relmax(c[0], fft_ref) < 1e-13


def _pipeline(ctx, wl, precision="fp64", obs=None, zero_value=1.0):
    N = wl.N if not isinstance(wl.N, dict) else None
    kw = {} if N is not None else wl.N
    ctx.plan(wl.curve, wl.W, wl.F, N=N, precision=precision, refine_tol=1e-14, refine_max=8,
             direction=wl.direction, **kw)
    psi, _, _ = ctx.solve_densities()
    obs = wl.obs if obs is None else obs
    V = ctx.eval_field(psi, obs, zero_value=zero_value)
    u = ctx.synthesize(wl.signal.f, wl.signal.t0, wl.signal.dt, wl.H, wl.tau0, V, wl.times)
    return u.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_pipeline_circle_pulse(ctx, precision):
    say("pipeline circle pulse", precision)
    wl = Wk.circle_pulse()
    u = _pipeline(ctx, wl, precision)
    ref = O.run(wl.curve, wl.W, wl.F, wl.N, wl.direction, wl.signal, wl.H, wl.tau0, wl.obs, wl.times)
    assert relmax(u, ref) < 1e-10


def test_pipeline_interior_identity(ctx):
    say("pipeline interior identity")
    sig = Wk.gaussian_pulse(t0=0.0, t1=30.0, dt=1 / 64, center=15.0, var2=1.0, freq=10.0)
    pts = np.array([[0.2, 0.1], [-0.5, 0.3], [0.0, -0.6]])
    wl = Wk.Workload("circ_int", Wk.circle(1.0), 24.0, 128, 64, direction=(0.6, 0.8), H=10.0, tau0=3.0,
                     signal=sig, obs=pts, times=np.linspace(0, 40, 81))
    u = _pipeline(ctx, wl)
    f = lambda t: np.exp(-(t - 15) ** 2) * np.cos(10 * t)
    exact = np.array([-f(wl.times - x @ np.array([0.6, 0.8])) for x in pts])
    assert np.max(np.abs(u - exact)) < 1e-9


def test_pipeline_kite_chirp_small(ctx):
    say("pipeline kite chirp small")
    W, F = 25.0, 64
    sig = Wk.chirp(300.0, np.pi / (4 * W))
    times = np.concatenate([np.linspace(0, 100, 64), np.linspace(200, 300, 64)])
    wl = Wk.Workload("kite_chirp_small", Wk.kite(), W, F, dict(ppw=10.0, n_min=64, n_mult=32, n_cap=4096),
                     direction=(1.0, 0.0), H=3.0, tau0=2.25, signal=sig, obs=Wk.ring(8, 3.0), times=times)
    u = _pipeline(ctx, wl)
    ref = O.run(wl.curve, W, F, wl.N, wl.direction, sig, wl.H, wl.tau0, wl.obs, times)
    assert relmax(u, ref) < 1e-10


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_run_one_call(ctx, fhw, precision):
    """fhw_run gives what the three calls give (same kernels, bit for bit) and
    the oracle's time samples; it refuses a plan of several curves."""
    say("fhw_run", precision)
    wl = Wk.circle_pulse()
    ref_sep = _pipeline(ctx, wl, precision)
    u, psi, V, resid, sweeps = ctx.run(wl.signal.f, wl.signal.t0, wl.signal.dt, wl.H, wl.tau0, wl.obs, wl.times)
    u = u.cpu().numpy()
    assert np.array_equal(u, ref_sep)
    ref = O.run(wl.curve, wl.W, wl.F, wl.N, wl.direction, wl.signal, wl.H, wl.tau0, wl.obs, wl.times)
    assert relmax(u, ref) < 1e-10
    if precision == "fp32_refine":
        assert np.all(resid <= 1e-14) and np.all(sweeps >= 1)
    ctx.plan([Wk.circle(1.0), Wk.kite()], wl.W, wl.F, N=64)
    with pytest.raises(fhw.FhwError) as e:
        ctx.run(wl.signal.f, wl.signal.t0, wl.signal.dt, wl.H, wl.tau0, wl.obs, wl.times)
    assert e.value.code == fhw.FHW_E_INVALID


def test_synthesis_tracking(ctx):
    """Active-partition tracking: a pulse sampled over a long silent range, a
    pure-delay spectrum; at track_tol = 1e-14 most (window, point) pairs
    leave the sum, the result equals the oracle's tracked synthesis and the
    untracked one within the tracking bound, and stays the exact delayed
    signal."""
    say("synthesis tracking")
    W, F, H, tau0 = 24.0, 128, 10.0, 3.0
    sig = Wk.gaussian_pulse(t0=0.0, t1=200.0, dt=1.0 / 64, center=15.0, var2=1.0, freq=10.0)
    ctx.plan(Wk.circle(1.0), W, F, N=64)
    dw = W / F
    omega_l = -W + dw * np.arange(2 * F)
    d = np.linspace(-1.0, 2.0, 6)
    Vh = np.exp(1j * omega_l[None, :] * d[:, None])
    V = torch.as_tensor(Vh, device="cuda")
    times = np.linspace(0.0, 190.0, 240)
    f = torch.as_tensor(sig.f, device="cuda")
    u0 = ctx.synthesize(f, sig.t0, sig.dt, H, tau0, V, times).cpu().numpy()
    p0, a0 = ctx.synth_active_pairs()
    u1 = ctx.synthesize(f, sig.t0, sig.dt, H, tau0, V, times, track_tol=1e-14).cpu().numpy()
    p1, a1 = ctx.synth_active_pairs()
    say("pairs", p1, "active untracked", a0, "tracked", a1)
    assert p0 == a0 == p1 and a1 < 0.5 * p1
    ks = O.window_indices(sig.t[0], sig.t[-1], H)
    act = np.zeros(len(ks), dtype=bool)
    for tt in times:
        act |= O.active_windows(tt, ks, H, tau0, dw)
    ks = ks[act]
    B = O.window_spectra(sig, H, ks, omega_l)
    ref1, _ = O.synthesize(Vh, B, ks, H, tau0, W, times, track_tol=1e-14)
    scale = np.max(np.abs(ref1))
    assert np.max(np.abs(u1 - ref1)) / scale < 1e-10
    assert np.max(np.abs(u1 - u0)) / scale < 1e-12
    exact = -np.exp(-(times[None, :] - d[:, None] - 15.0) ** 2) * np.cos(10.0 * (times[None, :] - d[:, None]))
    assert np.max(np.abs(u1 - exact)) < 1e-9


def test_synthesize_edge_cases(ctx, fhw):
    say("synthesize edges")
    wl = Wk.circle_pulse()
    ctx.plan(wl.curve, wl.W, wl.F, N=wl.N)
    psi, _, _ = ctx.solve_densities()
    V = ctx.eval_field(psi, wl.obs)
    # times far from the signal: no active window -> exactly zero
    u = ctx.synthesize(wl.signal.f, wl.signal.t0, wl.signal.dt, wl.H, wl.tau0, V, np.array([1e5, -1e5]))
    assert torch.count_nonzero(u).item() == 0
    # one time only, and an empty time list
    u1 = ctx.synthesize(wl.signal.f, wl.signal.t0, wl.signal.dt, wl.H, wl.tau0, V, np.array([5.0]))
    ref = O.run(wl.curve, wl.W, wl.F, wl.N, wl.direction, wl.signal, wl.H, wl.tau0, wl.obs, np.array([5.0]))
    assert relmax(u1.cpu().numpy(), ref) < 1e-10
    u0 = ctx.synthesize(wl.signal.f, wl.signal.t0, wl.signal.dt, wl.H, wl.tau0, V, np.zeros(0))
    assert u0.numel() == 0
    # 2F not a power of two
    ctx.plan(wl.curve, wl.W, 24, N=64)
    psi, _, _ = ctx.solve_densities()
    V = ctx.eval_field(psi, wl.obs)
    with pytest.raises(fhw.FhwError):
        ctx.synthesize(wl.signal.f, wl.signal.t0, wl.signal.dt, wl.H, wl.tau0, V, wl.times)


def test_densities_largest_N(ctx):
    """N = 4096, the largest order the plan accepts, one frequency: the
    small-batch solve keeps the whole vector in LDS (64 KiB beside its own
    17 KiB), in both precisions."""
    say("densities N = 4096, F = 1")
    curve, W, N = Wk.kite(), 40.0, 4096
    omega, kappa = O.frequency_grid(W, 1)
    eta = O.coupling(kappa)
    gm = O.geometry(curve, N)
    ref, _ = O.solve_density(O.assemble(gm, kappa[0], eta[0]), O.rhs_plane_wave(gm, kappa[0], eta[0], (1.0, 0.0)))
    for precision in ("fp64", "fp32_refine"):
        ctx.plan(curve, W, 1, N=N, precision=precision, refine_tol=1e-12, refine_max=10)
        psi, res, sw = ctx.solve_densities(compute_resid=True)
        err = relmax(psi.cpu().numpy(), ref)
        say("N = 4096", precision, "err", err, "resid", float(res[0]), "sweeps", int(sw[0]))
        assert err < 1e-11 and res[0] <= 1e-12


def test_single_frequency(ctx):
    say("F = 1")
    sig = Wk.gaussian_pulse()
    wl = Wk.Workload("circ_F1", Wk.circle(1.0), 8.0, 1, 64, H=4.0, tau0=0.0, signal=sig, obs=Wk.ring(3, 2.0),
                     times=np.linspace(0, 10, 5))
    u = _pipeline(ctx, wl)
    ref = O.run(wl.curve, wl.W, wl.F, wl.N, wl.direction, sig, wl.H, wl.tau0, wl.obs, wl.times)
    assert relmax(u, ref) < 1e-10


# ------------------------------------------------- several incidences (a5)
_INCS = [("plane", (1.0, 0.0)), ("plane", (0.6, -0.8)), ("point", (3.0, 0.5)), ("point", (-0.5, 2.9))]


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_incidences_kite_ragged(ctx, precision):
    """One factorization per frequency serves plane waves and exterior point
    sources; each density matches the oracle's own solve."""
    say("incidences kite ragged", precision)
    curve, W, F = Wk.kite(), 40.0, 6
    rule = dict(ppw=10.0, n_min=64, n_mult=32, n_cap=4096)
    Ns, off = ctx.plan(curve, W, F, precision=precision, refine_tol=1e-14, refine_max=8, **rule)
    psi, res, sw = ctx.solve_incidences(_INCS)
    assert psi.shape == (len(_INCS), int(off[-1]))
    _, kappa = O.frequency_grid(W, F)
    eta = O.coupling(kappa)
    P = psi.cpu().numpy()
    for j in range(F):
        gm = O.geometry(curve, int(Ns[j]))
        A = O.assemble(gm, kappa[j], eta[j])
        for q, (kind, v) in enumerate(_INCS):
            g = O.rhs_plane_wave(gm, kappa[j], eta[j], v) if kind == "plane" else O.rhs_point_source(gm, kappa[j], eta[j], v)
            ref, _ = O.solve_density(A, g)
            err = relmax(P[q, off[j]:off[j + 1]], ref)
            assert err < 1e-11, (j, q, err)
    if precision == "fp32_refine":
        assert np.all(res <= 1e-14)


def _many_incidences(n_plane=13, seed=11):
    """n_plane plane waves at seeded angles and point sources on a ring of
    radius 3.2 (outside the kite), interleaved so that every group of 8 mixes
    both kinds."""
    rng = np.random.default_rng(seed)
    ang = rng.uniform(0.0, 2.0 * np.pi, n_plane)
    planes = [("plane", (np.cos(a), np.sin(a))) for a in ang]
    points = [("point", (3.2 * np.cos(b), 3.2 * np.sin(b))) for b in (0.4, 1.3, 2.2, 3.1, 4.0, 4.9, 5.8)]
    out = []
    while planes or points:
        if planes:
            out.append(planes.pop(0))
        if planes:
            out.append(planes.pop(0))
        if points:
            out.append(points.pop(0))
    return out


def _check_many(psi, res, incs, curve, oms, Ns, off, precision, tag):
    """Every (frequency, incidence) density against the oracle's LAPACK solve:
    1e-11 in FP64; in FP32 + refinement within kappa_inf(A) sqrt(N) times the
    reported residual (and the residual within the tolerance asked)."""
    P = psi.cpu().numpy() if hasattr(psi, "cpu") else psi
    worst = 0.0
    for j, om in enumerate(oms):
        N = int(Ns[j])
        gm = O.geometry(curve, N)
        kappa = float(om)
        eta = float(O.coupling(np.array([kappa]))[0])
        A = O.assemble(gm, kappa, eta)
        cond = np.linalg.cond(A, np.inf)
        for q, (kind, v) in enumerate(incs):
            g = O.rhs_plane_wave(gm, kappa, eta, v) if kind == "plane" else O.rhs_point_source(gm, kappa, eta, v)
            ref, _ = O.solve_density(A, g)
            err = relmax(P[q, off[j]:off[j + 1]], ref)
            worst = max(worst, err)
            if precision == "fp64":
                assert err < 1e-11, (tag, j, q, err)
            else:
                assert res[q, j] <= 1e-13, (tag, j, q, res[q, j])
                assert err <= max(1e-11, cond * np.sqrt(N) * res[q, j]), (tag, j, q, err)
    say(tag, precision, "incidences", len(incs), "worst err vs oracle", worst)


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_many_incidences(fhw, precision):
    """More than one group of 8 incidences per factorization: 20 incidences
    (plane waves and exterior point sources, mixed within every group) on a
    ragged kite plan, through fhw_solve_incidences, then fhw_solve_cached on
    the resident factors (in another order), then fhw_solve_range on a plan
    of systems (two requests, 20 and 11 incidences)."""
    incs = _many_incidences()
    assert len(incs) == 20 and sum(k == "point" for k, _ in incs) == 7
    curve, W, F = Wk.kite(), 36.0, 5
    rule = dict(ppw=10.0, n_min=64, n_mult=32, n_cap=4096)
    omega, _ = O.frequency_grid(W, F)
    c = fhw.Context()
    try:
        say("many incidences: solve_incidences", precision)
        Ns, off = c.plan(curve, W, F, precision=precision, refine_tol=1e-13, refine_max=10, **rule)
        assert len(set(int(n) for n in Ns)) >= 3
        psi, res, sw = c.solve_incidences(incs)
        _check_many(psi, res, incs, curve, omega, Ns, off, precision, "solve_incidences")
        say("many incidences: solve_cached (reversed order)", precision)
        rev = incs[::-1]
        psi2, res2, _ = c.solve_cached(rev)
        _check_many(psi2, res2, rev, curve, omega, Ns, off, precision, "solve_cached")
        P, P2 = psi.cpu().numpy(), psi2.cpu().numpy()
        for q in range(len(incs)):
            assert relmax(P2[len(incs) - 1 - q], P[q]) < 1e-13, q
        say("many incidences: solve_range", precision)
        oms_a, oms_b = [omega[1], omega[3]], [omega[0], omega[2], omega[4]]
        systems = [(0, om, int(Ns[list(omega).index(om)])) for om in oms_a + oms_b]
        off_s = c.plan_systems([curve], systems, precision=precision, refine_tol=1e-13, refine_max=10)
        c.factor()
        pa, ra, _ = c.solve_range(0, 2, incs)
        _check_many(pa, ra, incs, curve, oms_a, [s[2] for s in systems[:2]], off_s[:3] - off_s[0], precision,
                    "solve_range A")
        inc_b = incs[4:15]
        pb, rb, _ = c.solve_range(2, 3, inc_b)
        _check_many(pb, rb, inc_b, curve, oms_b, [s[2] for s in systems[2:]], off_s[2:] - off_s[2], precision,
                    "solve_range B")
    finally:
        c.close()


def test_incidences_single_equals_densities(ctx):
    say("incidences: one plane wave = solve_densities")
    wl = Wk.circle_pulse()
    ctx.plan(wl.curve, wl.W, 16, N=wl.N, direction=(0.6, 0.8))
    psi1, _, _ = ctx.solve_densities()
    psi2, _, _ = ctx.solve_incidences([("plane", (0.6, 0.8))])
    assert relmax(psi2[0].cpu().numpy(), psi1.cpu().numpy()) < 1e-14


def test_point_source_interior_extinction(ctx):
    """Field of the point-source density inside the scatterer equals the free
    field of the source, G(x, r0) = (i/4) H0(kappa |x - r0|)."""
    say("point source interior extinction")
    curve, W, F, N = Wk.kite(), 12.0, 4, 256
    r0 = (2.5, 1.5)
    ctx.plan(curve, W, F, N=N)
    psi, res, _ = ctx.solve_incidences([("point", r0)], compute_resid=True)
    assert np.all(res < 1e-13)
    pts = Wk.interior_points(curve, 8, seed=7)
    V = ctx.eval_field(psi[0], pts, zero_value=0.0).cpu().numpy()
    _, kappa = O.frequency_grid(W, F)
    rho = np.hypot(pts[:, 0] - r0[0], pts[:, 1] - r0[1])
    for j in range(F):
        exact = 0.25j * special.hankel1(0, kappa[j] * rho)
        # the top frequency W is stored only as its conjugate at -W (index 0)
        Vj = V[:, F + 1 + j] if j < F - 1 else np.conj(V[:, 0])
        assert relmax(Vj, exact) < 1e-10
    assert np.all(V[:, F] == 0)


def test_pipeline_point_source(ctx):
    """Whole pipeline for an exterior point source vs the oracle's."""
    say("pipeline point source")
    sig = Wk.gaussian_pulse(t0=0.0, t1=20.0, dt=1 / 64, center=9.0, var2=2.0, freq=10.0)
    curve, W, F, N = Wk.circle(1.0), 24.0, 64, 96
    r0 = (2.0, 1.0)
    obs, times, H, tau0 = Wk.ring(6, 3.0), np.linspace(0, 30, 61), 6.0, 3.0
    ctx.plan(curve, W, F, N=N)
    psi, _, _ = ctx.solve_incidences([("point", r0)])
    V = ctx.eval_field(psi[0], obs, zero_value=0.0)
    u = ctx.synthesize(sig.f, sig.t0, sig.dt, H, tau0, V, times).cpu().numpy()
    ref = O.run(curve, W, F, N, (1.0, 0.0), sig, H, tau0, obs, times, incidence="point", r0=np.array(r0))
    assert relmax(u, ref) < 1e-10


def test_incidences_rejects(ctx, fhw):
    say("incidences: argument errors")
    ctx.plan(Wk.kite(), 10.0, 2, N=64)
    for bad in ([("point", (0.0, 0.0))],            # inside the kite
                [("plane", (1.0, 1.0))],            # not a unit vector
                [("plane", (float("nan"), 0.0))],
                [(7, (1.0, 0.0))],                  # unknown kind
                []):
        with pytest.raises(fhw.FhwError) as e:
            ctx.solve_incidences(bad)
        assert e.value.code == fhw.FHW_E_INVALID


def test_solve_cached(ctx, fhw):
    """Right-hand sides on resident factors equal a fresh solve; residency
    rules (no solve yet, FP64 residuals) are reported as FHW_E_STATE."""
    say("solve_cached")
    curve, W, F = Wk.kite(), 30.0, 4
    rule = dict(ppw=10.0, n_min=64, n_mult=32, n_cap=4096)
    incs = [("plane", (0.0, 1.0)), ("point", (2.5, -2.0))]
    for precision in ("fp64", "fp32_refine"):
        ctx.plan(curve, W, F, precision=precision, refine_tol=1e-14, refine_max=8, **rule)
        with pytest.raises(fhw.FhwError) as e:
            ctx.solve_cached(incs)
        assert e.value.code == fhw.FHW_E_STATE
        ref, _, _ = ctx.solve_incidences(incs)
        ctx.solve_densities()                        # factors stay resident
        got, res, _ = ctx.solve_cached(incs)
        assert relmax(got.cpu().numpy(), ref.cpu().numpy()) < 1e-14
        if precision == "fp32_refine":
            assert np.all(res <= 1e-14)
    ctx.plan(curve, W, F, precision="fp64", **rule)
    ctx.solve_densities(compute_resid=True)          # FP64 residuals re-assemble A over the factors
    with pytest.raises(fhw.FhwError) as e:
        ctx.solve_cached(incs)
    assert e.value.code == fhw.FHW_E_STATE


def test_chunked_plan_matches(fhw):
    """A small HBM budget splits the frequencies into several workspace
    chunks; the densities agree with a single-chunk plan to rounding (the
    panel kernel's sub-panel width follows the tallest matrix of a batch, so
    the batch composition changes the order of operations)."""
    say("chunked plan")
    curve, W, F = Wk.kite(), 40.0, 6
    rule = dict(ppw=10.0, n_min=64, n_mult=32, n_cap=4096)
    out = []
    for budget in (0, 16 << 20):
        c = fhw.Context(hbm_budget_bytes=budget)
        try:
            c.plan(curve, W, F, precision="fp32_refine", refine_tol=1e-14, refine_max=8, **rule)
            psi, _, _ = c.solve_densities()
            out.append(psi.cpu().numpy())
            if budget:
                with pytest.raises(fhw.FhwError) as e:
                    c.solve_cached([("plane", (1.0, 0.0))])
                assert e.value.code == fhw.FHW_E_STATE
        finally:
            c.close()
    assert relmax(out[1], out[0]) < 1e-13


# ---------------------------------------------- several curves in one plan
@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_plan_curves_star_batch(ctx, precision):
    """Seeded star curves planned together (one batch of ragged systems):
    every system's density and every curve's field against the oracle."""
    say("plan_curves star batch", precision)
    curves = Wk.star_pool(3, seed=0)
    W, F = 30.0, 8
    rule = dict(ppw=17.0, n_min=64, n_mult=32, n_cap=2048)
    Ns, off = ctx.plan(curves, W, F, precision=precision, refine_tol=1e-14, refine_max=8, **rule)
    assert len(Ns) == 3 * F and off[-1] == np.sum(Ns)
    psi, res, _ = ctx.solve_densities()
    P = psi.cpu().numpy()
    _, kappa = O.frequency_grid(W, F)
    eta = O.coupling(kappa)
    obs = Wk.ring(6, 3.0)
    for k, cv in enumerate(curves):
        Nk = O.discretization_sizes(kappa, O.curve_length(cv), **rule)
        assert np.array_equal(Ns[k * F:(k + 1) * F], Nk)
        V = ctx.eval_field(psi, obs, curve=k).cpu().numpy()
        for j in range(F):
            s = k * F + j
            gm = O.geometry(cv, int(Nk[j]))
            ref, _ = O.solve_density(O.assemble(gm, kappa[j], eta[j]), O.rhs_plane_wave(gm, kappa[j], eta[j], (1.0, 0.0)))
            assert relmax(P[off[s]:off[s + 1]], ref) < 1e-11, (k, j)
            Vj = V[:, F + 1 + j] if j < F - 1 else np.conj(V[:, 0])
            assert relmax(Vj, O.field(gm, ref, kappa[j], obs)) < 1e-11, (k, j)
    # incidences and argument checks apply to every curve
    psi2, _, _ = ctx.solve_incidences([("point", (4.0, 0.5))])
    for k, cv in enumerate(curves):
        s = k * F + F - 1
        gm = O.geometry(cv, int(Ns[s]))
        ref, _ = O.solve_density(O.assemble(gm, kappa[F - 1], eta[F - 1]),
                                 O.rhs_point_source(gm, kappa[F - 1], eta[F - 1], (4.0, 0.5)))
        assert relmax(psi2[0, off[s]:off[s + 1]].cpu().numpy(), ref) < 1e-11


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_band_plan(ctx, fhw, precision):
    """j_first > 0: the band (j_first + j) W/F, j = 1..F, solved for several
    plane waves; densities against the oracle; field and synthesis refuse it."""
    say("band plan", precision)
    curve, N, dw, j_first, F = Wk.kite(), 192, 1.0, 30, 6
    Ns, off = ctx.plan(curve, F * dw, F, N=N, precision=precision, refine_tol=1e-12, refine_max=10, j_first=j_first)
    dirs = [(1.0, 0.0), (0.0, 1.0), (0.6, -0.8)]
    psi, res, sw = ctx.solve_incidences([("plane", d) for d in dirs])
    psi = psi.cpu().numpy()
    gm = O.geometry(curve, N)
    for j in (0, F - 1):
        kappa = (j_first + j + 1) * dw
        eta = O.coupling(np.array([kappa]))[0]
        A = O.assemble(gm, kappa, eta)
        for q, d in enumerate(dirs):
            ref, _ = O.solve_density(A, O.rhs_plane_wave(gm, kappa, eta, d))
            assert relmax(psi[q, off[j]:off[j + 1]], ref) < 1e-11, (j, q)
    with pytest.raises(fhw.FhwError) as e:
        ctx.eval_field(torch.as_tensor(psi[0], device="cuda"), Wk.ring(4, 3.0))
    assert e.value.code == fhw.FHW_E_STATE


def test_workspace_reused_across_plans(fhw):
    """A stream of plans of different sizes and precisions on one context
    (the workspace kept and regrown) gives what fresh contexts give."""
    say("workspace reuse across plans")
    cases = [(Wk.kite(), 30.0, 8, 256, "fp32_refine"), (Wk.circle(1.0), 10.0, 4, 64, "fp64"),
             (Wk.kite(), 40.0, 12, 384, "fp32_refine"), (Wk.kite(), 20.0, 5, 128, "fp64")]
    c = fhw.Context()
    try:
        for curve, W, F, N, prec in cases:
            c.plan(curve, W, F, N=N, precision=prec, refine_tol=1e-12, refine_max=10)
            psi, _, _ = c.solve_densities()
            f = fhw.Context()
            try:
                f.plan(curve, W, F, N=N, precision=prec, refine_tol=1e-12, refine_max=10)
                psi_f, _, _ = f.solve_densities()
            finally:
                f.close()
            assert torch.equal(psi, psi_f), (W, F, N, prec)
    finally:
        c.close()


def _requests():
    """Four requests: (curve index, frequencies, N, incidences)."""
    return [(0, [31.0, 32.0, 33.0, 34.0], 192, [("plane", (1.0, 0.0)), ("plane", (0.0, 1.0)), ("plane", (0.6, -0.8))]),
            (1, [10.0, 11.5, 13.0], 256, [("plane", (-1.0, 0.0)), ("point", (3.5, 0.5))]),
            (2, [50.0, 51.0], 320, [("plane", (0.8, 0.6))] * 1 + [("plane", (np.cos(a), np.sin(a))) for a in (0.3, 1.1, 2.0, 2.9)]),
            # more than one group of 8 right-hand sides
            (1, [20.0, 21.0], 224, _many_incidences(n_plane=8, seed=5)[:12])]


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_requests_alone_and_in_the_mix(fhw, precision):
    """Requests of different curves, bands, N and right-hand sides factored in
    one batched plan (fhw_plan_systems + fhw_factor) and solved request by
    request (fhw_solve_range) give what each gives alone, and the oracle's
    densities."""
    say("requests alone vs in the mix", precision)
    curves = [Wk.star_pool(1, 3)[0], Wk.kite(), Wk.circle(1.2)]
    reqs = _requests()
    tol = 1e-12 if precision == "fp64" else 1e-10
    alone = []
    c = fhw.Context()
    try:
        for k, oms, N, inc in reqs:
            c.plan_systems(curves, [(k, om, N) for om in oms], precision=precision)
            c.factor()
            psi, res, sw = c.solve_range(0, len(oms), inc)
            alone.append(psi.cpu().numpy())
        systems = [(k, om, N) for k, oms, N, _ in reqs for om in oms]
        off = c.plan_systems(curves, systems, precision=precision)
        c.factor()
        s0 = 0
        for (k, oms, N, inc), a in zip(reqs, alone):
            psi, res, sw = c.solve_range(s0, len(oms), inc)
            psi = psi.cpu().numpy()
            err = relmax(psi, a)
            say("request", k, "N", N, "mix vs alone", err)
            assert err < tol
            if precision == "fp32_refine":
                assert np.all(res <= 1e-12)
            # the oracle on the first frequency of the request, every incidence
            gm = O.geometry(curves[k], N)
            kappa = oms[0]
            eta = O.coupling(np.array([kappa]))[0]
            A = O.assemble(gm, kappa, eta)
            for q, (kind, v) in enumerate(inc):
                g = O.rhs_plane_wave(gm, kappa, eta, v) if kind == "plane" else O.rhs_point_source(gm, kappa, eta, v)
                ref, _ = O.solve_density(A, g)
                err = relmax(psi[q, :N], ref)
                if precision == "fp64":
                    assert err < 1e-11, (k, q, err)
                else:
                    # ||d psi||_inf / ||psi||_inf <= kappa_inf(A) sqrt(N) ||r||_2 / ||g||_2
                    assert err <= max(1e-11, np.linalg.cond(A, np.inf) * np.sqrt(N) * res[q, 0]), (k, q, err)
            s0 += len(oms)
        with pytest.raises(fhw.FhwError) as e:
            c.eval_field(torch.zeros(int(off[-1]), dtype=torch.complex128, device="cuda"), Wk.ring(4, 3.0))
        assert e.value.code == fhw.FHW_E_STATE
        with pytest.raises(fhw.FhwError) as e:
            c.solve_range(len(systems) - 1, 2, [("plane", (1.0, 0.0))])
        assert e.value.code == fhw.FHW_E_INVALID
        c.plan_systems(curves, systems[:2], precision=precision)
        with pytest.raises(fhw.FhwError) as e:
            c.solve_range(0, 1, [("plane", (1.0, 0.0))])
        assert e.value.code == fhw.FHW_E_STATE
    finally:
        c.close()


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_factorization_graph_replays(ctx, precision):
    """The factorization runs as one captured graph when the stage timers are
    off: replayed several times, with eager work and synchronizations between
    the replays, every result equals the eager (timed, launch by launch) one."""
    say("factorization graph replays", precision)
    ctx.plan(Wk.kite(), 30.0, 12, precision=precision, refine_tol=1e-12, refine_max=10,
             ppw=10.0, n_min=64, n_mult=32, n_cap=4096)
    ctx.profile(True)
    psi_e, res_e, _ = ctx.solve_densities()
    ctx.profile(False)
    psi_e = psi_e.clone()
    obs = Wk.ring(8, 3.0)
    for rep in range(4):
        psi, res, _ = ctx.solve_densities()
        V = ctx.eval_field(psi, obs)
        x = torch.ones(1 << 20, dtype=torch.float64, device="cuda").cumsum(0)
        torch.cuda.synchronize()
        assert torch.equal(psi, psi_e), rep
        assert np.array_equal(res, res_e)
        assert float(x[-1]) == float(1 << 20) and torch.isfinite(V).all()


def test_budget_too_small(fhw):
    """A workspace budget below one frequency's needs is FHW_E_NOMEM at plan
    time, and the context stays usable."""
    say("budget too small")
    c = fhw.Context(hbm_budget_bytes=4 << 20)
    try:
        with pytest.raises(fhw.FhwError) as e:
            c.plan(Wk.kite(), 40.0, 4, N=1024)          # one N = 1024 matrix alone is 16 MiB
        assert e.value.code == fhw.FHW_E_NOMEM
        c.plan(Wk.kite(), 10.0, 2, N=64)
        psi, _, _ = c.solve_densities()
        assert torch.isfinite(torch.view_as_real(psi)).all()
    finally:
        c.close()
