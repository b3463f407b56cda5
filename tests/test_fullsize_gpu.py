"""Parity at full size, in FP32 LU + FP64 refinement to 1e-12 and in FP64:
  * kite_N1024_F1024: the solve-throughput workload, planned exactly as the
    benchmark plans it: kite, N = 1024 at each of 1024 frequencies on (0, 69];
  * kite_chirp_F512_W200: kite, 512 frequencies on (0, 200] with N from 10
    points per wavelength (64 .. 2976), the paper's chirp;
both with one plane-wave direction, 256 points on the radius-3 ring and 1024
times reaching T = 1e4.

The oracle cannot redo all 1024 solves inside a test, so:
  * densities and fields are compared at sampled frequencies, each solved by
    the oracle on its own;
  * time samples are compared with oracle values written by
    tests/golden/make_golden.py (4 of the 256 points, all times);
  * the synthesis alone runs on a pure-delay spectrum V = exp(i w d_r), whose
    time-domain field is the delayed boundary signal -f(t - d_r) in closed form;
  * points inside the kite see the incident signal exactly (extinction).
Tolerances: FP64 densities 1e-11 (relative, max norm); FP32+refinement
densities kappa_2(A) times the reported residual; time samples 1e-10 relative
to the largest sample.
"""
import json
import os

import numpy as np
import pytest
import torch
from scipy import special

import oracle as O
import workloads as Wk

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
REFINE_TOL = 1e-12
WORKLOADS = {"kite_n1024": (Wk.kite_n1024, [0, 255, 511, 767, 1023]),
             "kite_chirp": (Wk.kite_chirp, [0, 170, 341, 511])}


def say(*a):
    print("CASE", *a, flush=True)


def relmax(a, b):
    a = np.asarray(a); b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


@pytest.fixture(scope="module")
def fhw():
    from paper_1807_02718_amd import fhw as m
    return m


def _plan_kw(wl):
    return dict(N=wl.N) if not isinstance(wl.N, dict) else dict(wl.N)


def _sizes(wl):
    omega, kappa = O.frequency_grid(wl.W, wl.F)
    if isinstance(wl.N, dict):
        return kappa, O.discretization_sizes(kappa, O.curve_length(wl.curve), **wl.N)
    return kappa, np.full(wl.F, wl.N)


@pytest.fixture(scope="module", params=list(WORKLOADS))
def wl(request):
    make, sampled = WORKLOADS[request.param]
    w = make()
    w.extra["sampled"] = sampled
    return w


@pytest.fixture(scope="module")
def oracle_sampled(wl):
    """Oracle densities, fields and condition numbers at the sampled
    frequencies."""
    kappa, Ns = _sizes(wl)
    eta = O.coupling(kappa)
    out = {}
    for j in wl.extra["sampled"]:
        gm = O.geometry(wl.curve, int(Ns[j]))
        A = O.assemble(gm, kappa[j], eta[j])
        g = O.rhs_plane_wave(gm, kappa[j], eta[j], wl.direction)
        psi, _ = O.solve_density(A, g)
        V = O.field(gm, psi, kappa[j], wl.obs)
        out[j] = dict(A=A, g=g, psi=psi, V=V, cond=float(np.linalg.cond(A)))
    return out


@pytest.fixture(scope="module", params=["fp32_refine", "fp64"])
def gpu_run(request, fhw, wl):
    precision = request.param
    say("full-size", wl.name, precision)
    ctx = fhw.Context()
    Ns, off = ctx.plan(wl.curve, wl.W, wl.F, precision=precision, refine_tol=REFINE_TOL,
                       refine_max=10, direction=wl.direction, **_plan_kw(wl))
    psi, resid, sweeps = ctx.solve_densities(compute_resid=True)
    V = ctx.eval_field(psi, wl.obs, zero_value=1.0)
    f = torch.as_tensor(wl.signal.f, device=psi.device)
    u = ctx.synthesize(f, wl.signal.t0, wl.signal.dt, wl.H, wl.tau0, V, wl.times)
    res = dict(precision=precision, Ns=np.asarray(Ns), off=np.asarray(off), resid=resid, sweeps=sweeps,
               psi={j: psi[int(off[j]):int(off[j + 1])].cpu().numpy() for j in wl.extra["sampled"]},
               psi_all=psi.cpu().numpy(),
               V=V.cpu().numpy(), u=u.cpu().numpy(), ctx=ctx)
    yield res
    ctx.close()


def test_fullsize_densities_sampled(gpu_run, oracle_sampled, wl):
    prec = gpu_run["precision"]
    assert np.array_equal(gpu_run["Ns"], _sizes(wl)[1])
    if prec == "fp32_refine":
        assert np.max(gpu_run["resid"]) <= REFINE_TOL
    for j in wl.extra["sampled"]:
        o = oracle_sampled[j]
        p = gpu_run["psi"][j]
        err = relmax(p, o["psi"])
        err2 = float(np.linalg.norm(p - o["psi"]) / np.linalg.norm(o["psi"]))
        # residual of the GPU density against the oracle's matrix and data
        r_o = float(np.linalg.norm(o["g"] - o["A"] @ p) / np.linalg.norm(o["g"]))
        say(wl.name, prec, "freq", j, "N", len(p), "cond", round(o["cond"], 2), "err_inf", err, "err_2", err2, "resid(oracle A)", r_o,
            "sweeps", int(gpu_run["sweeps"][j]))
        if prec == "fp64":
            assert err < 1e-11
        else:
            assert r_o <= 1.5 * REFINE_TOL
            # ||d psi|| <= kappa_2 ||r|| / ||g|| ||psi|| (plus the FP64 floor)
            assert err2 <= 1.1 * o["cond"] * r_o + 1e-13


def test_fullsize_field_sampled(gpu_run, oracle_sampled, wl):
    prec = gpu_run["precision"]
    F = wl.F
    V = gpu_run["V"]
    assert V.shape == (len(wl.obs), 2 * F)
    kappa, Ns = _sizes(wl)
    for j in wl.extra["sampled"]:
        o = oracle_sampled[j]
        # omega_{j+1} sits at grid index F + 1 + j; the top frequency W is
        # held only through its conjugate at -W (index 0) on [-W, W)
        if F + 1 + j < 2 * F:
            Vg = V[:, F + 1 + j]
            assert np.array_equal(V[:, F - 1 - j], np.conj(Vg))   # Hermitian extension
        else:
            Vg = np.conj(V[:, 0])
        err = relmax(Vg, o["V"])
        say(wl.name, prec, "field freq", j, "err", err)
        if prec == "fp64":
            assert err < 1e-11
        else:
            # the field is a fixed linear functional of the density:
            # |dV_r| <= ||w_r||_2 ||d psi||_2 with w_r = (pi/n) (i/4) H0 |x'|
            n_j = int(Ns[j])
            gm = O.geometry(wl.curve, n_j)
            d = np.hypot(wl.obs[:, None, 0] - gm["x"][None, :, 0], wl.obs[:, None, 1] - gm["x"][None, :, 1])
            w = (np.pi / (n_j // 2)) * 0.25 * np.abs(special.hankel1(0, kappa[j] * d)) * gm["speed"][None, :]
            bound = np.linalg.norm(w, axis=1) * np.linalg.norm(gpu_run["psi"][j] - o["psi"])
            assert np.all(np.abs(Vg - o["V"]) <= 1.1 * bound + 1e-13 * np.max(np.abs(o["V"])))
    assert np.all(V[:, F] == 1.0)


def _subset_errors(name, psi_all, off, resid):
    """Sampled densities of the subset written by
    tests/golden/make_golden_subsets.py against the GPU's: per system
    max |d psi| / max |psi| over the 64 samples, with the system's N, the
    oracle's condition estimate and the GPU's residual."""
    gold = np.load(os.path.join(HERE, "golden", f"{name}_psi_sub16.npz"))
    rows = []
    for q, s in enumerate(gold["system"]):
        N = int(gold["N"][q])
        assert int(off[s + 1] - off[s]) == N, (s, N)
        idx = np.round(np.linspace(0, N - 1, gold["psi"].shape[1])).astype(np.int64)
        p = psi_all[int(off[s]) + idx]
        err = float(np.max(np.abs(p - gold["psi"][q])) / gold["psi_max"][q])
        rows.append((int(s), N, err, float(gold["cond_inf"][q]), float(resid[s])))
    return rows


def test_fullsize_subset_per_frequency(gpu_run, wl):
    """The precision configuration's error against the FP64 oracle at every
    16th frequency of the kite workload with N from 10 points per wavelength
    (32 frequencies, N = 96 .. 2976), both precisions: FP64 within 1e-11;
    FP32 LU + refinement within kappa_inf(A) sqrt(N) times its residual."""
    if wl.name != "kite_chirp_F512_W200":
        pytest.skip("the every-16th-frequency subset is written for the kite workload with N from the rule")
    prec = gpu_run["precision"]
    rows = _subset_errors("kite_chirp", gpu_run["psi_all"], gpu_run["off"], gpu_run["resid"])
    for s, N, err, cond, r in rows:
        say(wl.name, prec, "freq", s, "N", N, "err", "%.2e" % err, "cond_inf", round(cond, 1), "resid", "%.1e" % r)
        if prec == "fp64":
            assert err < 1e-11, (s, err)
        else:
            assert r <= REFINE_TOL and err <= max(1e-11, cond * np.sqrt(N) * r), (s, err)
    say(wl.name, prec, "subset of", len(rows), "frequencies: max err", max(e for _, _, e, _, _ in rows))


def test_star_batch_subset_vs_oracle(fhw):
    """The batching configuration at full size (64 seeded star curves x 256
    frequencies on (0, 120], N = 64 .. 2048 from 17 points per wavelength,
    FP64; about 384 GB of matrices, so the plan runs in more than one
    workspace chunk): every 16th system against the oracle's densities, 1e-11
    relative."""
    sb = Wk.star_batch()
    say("star batch full size, fp64")
    ctx = fhw.Context()
    try:
        Ns, off = ctx.plan(sb["curves"], sb["W"], sb["F"], precision="fp64", direction=sb["direction"], **sb["rule"])
        assert int(Ns.max()) == 2048 and int(Ns.min()) == 64
        assert float(np.sum(16.0 * Ns.astype(np.float64) ** 2)) > torch.cuda.get_device_properties(0).total_memory
        psi, _, _ = ctx.solve_densities()
        psi_all = psi.cpu().numpy()
    finally:
        ctx.close()
    rows = _subset_errors("star_batch", psi_all, off, np.zeros(len(Ns)))
    worst = max(rows, key=lambda r: r[2])
    say("star batch subset:", len(rows), "systems, N", min(r[1] for r in rows), "..", max(r[1] for r in rows),
        "max err", worst[2], "at system", worst[0])
    assert all(e < 1e-11 for _, _, e, _, _ in rows), worst


def test_fullsize_time_samples_vs_oracle(gpu_run, wl):
    meta = json.load(open(os.path.join(HERE, "golden", f"{wl.name}_u_sample.json")))
    ref = np.load(os.path.join(HERE, "golden", f"{wl.name}_u_sample.npy"))
    assert meta["workload"] == wl.name and ref.shape == (len(meta["obs_index"]), len(wl.times))
    u = gpu_run["u"][meta["obs_index"]]
    err = relmax(u, ref)
    per_t = np.max(np.abs(u - ref), axis=0) / np.max(np.abs(ref))
    say(wl.name, gpu_run["precision"], "time samples vs oracle (4 points x 1024 times)", err, "max|u|",
        float(np.max(np.abs(ref))), "per-time error quartiles", np.percentile(per_t, [50, 90, 100]).tolist())
    assert err < 1e-10
    assert np.all(np.isfinite(gpu_run["u"]))


def test_fullsize_synthesis_delay(fhw):
    """Synthesis of a pure delay V(r, w) = exp(i w d_r) on the full DFT grid:
    the field is a(t - d_r) = -f(t - d_r), and the oracle's synthesis from the
    same spectrum agrees on a sample of points."""
    say("full-size synthesis, delay spectrum")
    wl = Wk.kite_n1024()
    ctx = fhw.Context()
    try:
        ctx.plan(wl.curve, wl.W, wl.F, N=wl.N)
        Nr = len(wl.obs)
        d = np.linspace(-3.0, 5.0, Nr)
        dw = wl.W / wl.F
        omega_l = -wl.W + dw * np.arange(2 * wl.F)
        Vh = np.exp(1j * omega_l[None, :] * d[:, None])
        V = torch.as_tensor(Vh, device="cuda")
        f = torch.as_tensor(wl.signal.f, device="cuda")
        u = ctx.synthesize(f, wl.signal.t0, wl.signal.dt, wl.H, wl.tau0, V, wl.times).cpu().numpy()
    finally:
        ctx.close()
    exact = -Wk.chirp_value(wl.times[None, :] - d[:, None], 1.0e4 + 5.0, rate=16000.0)
    err_exact = float(np.max(np.abs(u - exact)))
    # the oracle's synthesis on 8 of the points
    sel = np.arange(0, Nr, Nr // 8)
    t = wl.signal.t
    ks = O.window_indices(t[0], t[-1], wl.H)
    act = np.zeros(len(ks), dtype=bool)
    for tt in wl.times:
        act |= O.active_windows(tt, ks, wl.H, wl.tau0, dw)
    ks = ks[act]
    B = O.window_spectra(wl.signal, wl.H, ks, omega_l)
    ref, _ = O.synthesize(Vh[sel], B, ks, wl.H, wl.tau0, wl.W, wl.times)
    err_o = relmax(u[sel], ref)
    say("delay: |u - exact|", err_exact, "vs oracle", err_o, "windows", len(ks))
    assert err_o < 1e-10
    assert err_exact < 1e-9


def test_fullsize_interior_extinction(fhw):
    """Points inside the kite: the scattered field cancels the incident one, so
    u(x, t) = -f(t - p.x) (plane wave, direction p)."""
    say("full-size interior extinction")
    wl = Wk.kite_n1024()
    pts = Wk.interior_points(wl.curve, 16, seed=5)
    ctx = fhw.Context()
    try:
        ctx.plan(wl.curve, wl.W, wl.F, N=wl.N, precision="fp32_refine", refine_tol=REFINE_TOL, refine_max=10,
                 direction=wl.direction)
        psi, _, _ = ctx.solve_densities()
        V = ctx.eval_field(psi, pts, zero_value=1.0)
        f = torch.as_tensor(wl.signal.f, device=psi.device)
        u = ctx.synthesize(f, wl.signal.t0, wl.signal.dt, wl.H, wl.tau0, V, wl.times).cpu().numpy()
    finally:
        ctx.close()
    p = np.asarray(wl.direction)
    exact = -Wk.chirp_value(wl.times[None, :] - (pts @ p)[:, None], 1.0e4 + 5.0, rate=16000.0)
    err = float(np.max(np.abs(u - exact)))
    say("interior extinction max error", err)
    assert err < 1e-9


def test_fullsize_uniform_synthesis(fhw):
    """The fast scaled convolution in the configuration the uniform-grid
    benchmark times (kite workload's band: F = 1024 so L = 4096 and chirp-z
    length 8192; 256 points; 16384 samples at pi/(4W) from t = 9000), on a
    pure-delay spectrum: against the oracle's written-out approximation on a
    sample (4 points x 64 grid times), the direct GPU sum on every sample,
    and the delayed chirp -f(t - d_r)."""
    say("full-size uniform synthesis")
    wl = Wk.kite_n1024()
    ctx = fhw.Context()
    Nr = len(wl.obs)
    d = np.linspace(-3.0, 5.0, Nr)
    dw = wl.W / wl.F
    omega_l = -wl.W + dw * np.arange(2 * wl.F)
    Vh = np.exp(1j * omega_l[None, :] * d[:, None])
    t_first, t_step, n_t = 9000.0, np.pi / (4.0 * wl.W), 16384
    times = t_first + t_step * np.arange(n_t)
    try:
        ctx.plan(wl.curve, wl.W, wl.F, N=wl.N)
        V = torch.as_tensor(Vh, device="cuda")
        f = torch.as_tensor(wl.signal.f, device="cuda")
        u = ctx.synthesize_uniform(f, wl.signal.t0, wl.signal.dt, wl.H, wl.tau0, V, t_first, t_step,
                                   n_t).cpu().numpy()
        ud = ctx.synthesize(f, wl.signal.t0, wl.signal.dt, wl.H, wl.tau0, V, times).cpu().numpy()
    finally:
        ctx.close()
    rows = np.arange(0, Nr, Nr // 4)
    cols = np.sort(np.random.default_rng(2).choice(2000, 64, replace=False))
    t = wl.signal.t
    ks = O.window_indices(t[0], t[-1], wl.H)
    act = np.zeros(len(ks), dtype=bool)
    for tt in times[cols]:
        act |= O.active_windows(tt, ks, wl.H, wl.tau0, dw)
    ks = ks[act]
    B = O.window_spectra(wl.signal, wl.H, ks, omega_l)
    ref = O.synthesize_uniform(Vh[rows], B, ks, wl.H, wl.tau0, wl.W, t_first, t_step, n_t, 4 * wl.F, t_index=cols)
    exact = -Wk.chirp_value(times[None, :] - d[:, None], 1.0e4 + 5.0, rate=16000.0)
    err_o = relmax(u[np.ix_(rows, cols)], ref)
    err_d = float(np.max(np.abs(u - ud)) / np.max(np.abs(ud)))
    err_x = float(np.max(np.abs(u - exact)))
    say("uniform: vs oracle", err_o, "vs direct", err_d, "vs exact", err_x, "windows in the sample", len(ks))
    assert err_o < 1e-10
    assert err_d < 1e-10
    assert err_x < 1e-9
