"""The serving component (fhw_server_*) through the C ABI: requests of
different scatterers, bands, N and right-hand sides (more than 8 for some)
submitted together to a server of two worker slots give what each gives
alone (fhw_plan_systems + fhw_factor + fhw_solve_range on its own), and the
oracle's densities on the first frequency of every request; a full queue
refuses with FHW_E_BUSY and the admitted requests still complete."""
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


def _incs(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n):
        if q % 4 == 3:
            b = rng.uniform(0.0, 2.0 * np.pi)
            out.append(("point", (3.4 * np.cos(b), 3.4 * np.sin(b))))
        else:
            a = rng.uniform(0.0, 2.0 * np.pi)
            out.append(("plane", (np.cos(a), np.sin(a))))
    return out


CURVES = [Wk.star_pool(1, 3)[0], Wk.kite(), Wk.circle(1.2), Wk.star_pool(2, 7)[1]]
REQUESTS = [(0, [31.0, 32.0, 33.0], 192, _incs(3, 1)),
            (1, [10.0, 11.5], 256, _incs(12, 2)),
            (2, [50.0, 51.0, 52.0, 53.0], 320, _incs(1, 3)),
            (3, [5.0], 96, _incs(9, 4)),
            (1, [20.0, 21.0, 22.0], 224, _incs(5, 5)),
            (0, [40.0], 288, _incs(17, 6))]


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_server_requests_alone_and_in_the_mix(fhw, precision):
    say("server: requests alone vs in the mix", precision)
    alone = []
    c = fhw.Context()
    try:
        for k, oms, N, inc in REQUESTS:
            c.plan_systems(CURVES, [(k, om, N) for om in oms], precision=precision, refine_tol=1e-13)
            c.factor()
            psi, res, _ = c.solve_range(0, len(oms), inc)
            alone.append((psi.cpu().numpy(), res))
    finally:
        c.close()
    srv = fhw.Server(CURVES, precision=precision, refine_tol=1e-13, slots=2)
    try:
        subs = [srv.submit(k, oms, N, inc) for k, oms, N, inc in REQUESTS]
        for (t, psi, res, sw), (k, oms, N, inc), (pa, ra) in zip(subs, REQUESTS, alone):
            assert srv.poll(t, wait=True) == fhw.FHW_OK
            got = psi.cpu().numpy()
            err = relmax(got, pa)
            say("request curve", k, "N", N, "rhs", len(inc), "server vs alone", err)
            assert err < (1e-12 if precision == "fp64" else 1e-10)
            if precision == "fp32_refine":
                assert np.all(res <= 1e-13) and np.all(sw >= 1)
            # the oracle at the request's first frequency, every incidence
            gm = O.geometry(CURVES[k], N)
            kappa = oms[0]
            eta = float(O.coupling(np.array([kappa]))[0])
            A = O.assemble(gm, kappa, eta)
            cond = np.linalg.cond(A, np.inf)
            for q, (kind, v) in enumerate(inc):
                g = O.rhs_plane_wave(gm, kappa, eta, v) if kind == "plane" else O.rhs_point_source(gm, kappa, eta, v)
                ref, _ = O.solve_density(A, g)
                e = relmax(got[q, :N], ref)
                if precision == "fp64":
                    assert e < 1e-11, (k, q, e)
                else:
                    assert e <= max(1e-11, cond * np.sqrt(N) * res[q, 0]), (k, q, e)
        st = srv.stats()
        say("server stats", st)
        assert st["done"] == len(REQUESTS) and st["refused"] == 0 and st["rounds"] >= 1
    finally:
        srv.close()


def test_server_busy_when_the_queue_is_full(fhw):
    """One slot and a queue limit of one byte (a request is admitted only
    while nothing waits): a burst of submissions is partly refused
    (FHW_E_BUSY); every admitted request completes with its densities equal
    to the request solved alone."""
    say("server: admission refusal")
    k, oms, N, inc = 1, [12.0, 13.0, 14.0, 15.0], 320, _incs(4, 9)
    c = fhw.Context()
    try:
        c.plan_systems(CURVES, [(k, om, N) for om in oms], precision="fp64")
        c.factor()
        ref = c.solve_range(0, len(oms), inc)[0].cpu().numpy()
    finally:
        c.close()
    srv = fhw.Server(CURVES, precision="fp64", slots=1, queue_limit_bytes=1)
    try:
        admitted, busy = [], 0
        for _ in range(20):
            try:
                admitted.append(srv.submit(k, oms, N, inc))
            except fhw.FhwError as e:
                assert e.code == fhw.FHW_E_BUSY
                busy += 1
        for t, psi, _, _ in admitted:
            assert srv.poll(t, wait=True) == fhw.FHW_OK
            assert relmax(psi.cpu().numpy(), ref) < 1e-12
        st = srv.stats()
        say("admitted", len(admitted), "refused", busy, "stats", st)
        assert busy >= 1 and st["refused"] == busy and st["done"] == len(admitted)
        with pytest.raises(fhw.FhwError) as e:
            srv.poll(admitted[0][0])      # reported once, then forgotten
        assert e.value.code == fhw.FHW_E_INVALID
    finally:
        srv.close()


def test_server_factor_cache(fhw):
    """A request repeated after its round (same curve, frequencies and N, new
    right-hand sides) is served from the slot's resident factors: no new
    factorization, and the densities equal those of a fresh solve."""
    say("server: factor cache")
    k, oms, N = 0, [25.0, 26.0, 27.0], 256
    inc1, inc2 = _incs(3, 11), _incs(10, 12)
    c = fhw.Context()
    try:
        c.plan_systems(CURVES, [(k, om, N) for om in oms], precision="fp32_refine", refine_tol=1e-13)
        c.factor()
        ref2 = c.solve_range(0, len(oms), inc2)[0].cpu().numpy()
    finally:
        c.close()
    srv = fhw.Server(CURVES, precision="fp32_refine", refine_tol=1e-13, slots=1)
    try:
        t1, *_ = srv.submit(k, oms, N, inc1)
        assert srv.poll(t1, wait=True) == fhw.FHW_OK
        s1 = srv.stats()
        t2, psi2, res2, _ = srv.submit(k, oms, N, inc2)
        assert srv.poll(t2, wait=True) == fhw.FHW_OK
        s2 = srv.stats()
        say("stats after the first", s1, "after the repeat", s2)
        assert s2["cache_hits"] == s1["cache_hits"] + 1 and s2["systems"] == s1["systems"]
        assert relmax(psi2.cpu().numpy(), ref2) < 1e-10 and np.all(res2 <= 1e-13)
    finally:
        srv.close()
