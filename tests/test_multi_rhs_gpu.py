"""Several right-hand sides per factorization on batches wide enough for the
group kernels (k_lu_solve_multi: more than 256 matrices; k_residual_multi:
at least 512 row blocks), which read each matrix once for all vectors of a
group instead of once per vector.  20 incidences (plane waves and exterior
point sources, mixed in every group of 8) on the kite at 520 frequencies,
both precisions, through fhw_solve_incidences, against the oracle's LAPACK
solves at sampled frequencies and against the same incidences solved one at
a time (single-vector kernels); plus N = 2560 (two vectors per workgroup: four
would outgrow the LDS) on a band of 264 frequencies with the FP64 residuals of
fhw_solve_incidences."""
import numpy as np
import pytest

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


def incidences(n_plane=13, seed=11):
    rng = np.random.default_rng(seed)
    planes = [("plane", (np.cos(a), np.sin(a))) for a in rng.uniform(0.0, 2.0 * np.pi, n_plane)]
    points = [("point", (3.2 * np.cos(b), 3.2 * np.sin(b))) for b in (0.4, 1.3, 2.2, 3.1, 4.0, 4.9, 5.8)]
    out = []
    while planes or points:
        out += planes[:2] + points[:1]
        planes, points = planes[2:], points[1:]
    return out


def oracle_check(P, res, incs, curve, omega, N, js, precision, tag):
    worst = 0.0
    for j in js:
        gm = O.geometry(curve, N)
        kappa = float(omega[j])
        eta = float(O.coupling(np.array([kappa]))[0])
        A = O.assemble(gm, kappa, eta)
        cond = np.linalg.cond(A, np.inf)
        for q, (kind, v) in enumerate(incs):
            g = O.rhs_plane_wave(gm, kappa, eta, v) if kind == "plane" else O.rhs_point_source(gm, kappa, eta, v)
            ref, _ = O.solve_density(A, g)
            err = relmax(P[q, j * N:(j + 1) * N], ref)
            worst = max(worst, err)
            if precision == "fp64":
                assert err < 1e-11, (tag, j, q, err)
            else:
                assert res[q, j] <= 1e-13, (tag, j, q, res[q, j])
                assert err <= max(1e-11, cond * np.sqrt(N) * res[q, j]), (tag, j, q, err)
    say(tag, precision, "worst err vs oracle", worst)


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_group_kernels_wide_batch(fhw, precision):
    incs = incidences()
    curve, W, F, N = Wk.kite(), 52.0, 520, 64
    omega, _ = O.frequency_grid(W, F)
    c = fhw.Context()
    try:
        say("group kernels: kite N", N, "F", F, precision, "incidences", len(incs))
        c.plan(curve, W, F, N=N, precision=precision, refine_tol=1e-13, refine_max=10)
        psi, res, sw = c.solve_incidences(incs)
        P = psi.cpu().numpy()
        one = np.stack([c.solve_cached([inc])[0][0].cpu().numpy() for inc in incs[:9]])
    finally:
        c.close()
    e1 = relmax(P[:9], one)
    say("group vs one at a time (9 incidences)", precision, e1)
    assert e1 < (1e-13 if precision == "fp64" else 1e-11)
    oracle_check(P, res, incs, curve, omega, N, [0, 37, 259, 260, 518, 519], precision, "wide batch")
    if precision == "fp32_refine":
        assert np.all(res <= 1e-13) and np.all(sw >= 1)


def test_group_kernels_two_per_workgroup_fp64_residuals(fhw):
    """N = 2560 puts two vectors in each solve workgroup (four would need
    more LDS than a workgroup may have); FP64 residuals (compute_resid) go
    through the group residual kernel."""
    incs = incidences(n_plane=7, seed=3)[:9]
    curve, W, F, N = Wk.kite(), 30.0, 264, 2560
    omega, _ = O.frequency_grid(W, F)
    c = fhw.Context()
    try:
        say("group kernels: kite N", N, "F", F, "fp64 with residuals")
        c.plan(curve, W, F, N=N, precision="fp64")
        psi, res, _ = c.solve_incidences(incs, compute_resid=True)
        P = psi.cpu().numpy()
    finally:
        c.close()
    say("fp64 residuals: max", float(res.max()))
    assert np.all(res < 1e-12)
    oracle_check(P, res, incs, curve, omega, N, [0, 263], "fp64", "two per workgroup")
