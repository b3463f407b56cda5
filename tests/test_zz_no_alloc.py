"""The allocation-free solve entry point (fhw_solve_range_noalloc) against the
entry point it varies (fhw_solve_range), through the C ABI: two calls in a
row on the same resident factors, the second with fewer systems and fewer
incidences, in both precisions; results equal to the last bit (the same
kernels run on the same data), and the size limit refused."""
import numpy as np
import pytest
import torch

import workloads as Wk

pytestmark = pytest.mark.gpu


def say(*a):
    print("CASE", *a, flush=True)


@pytest.fixture(scope="module")
def fhw():
    from paper_1807_02718_amd import fhw as m
    return m


def _incidences(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for q in range(n):
        if q % 3 == 2:
            b = rng.uniform(0.0, 2.0 * np.pi)
            out.append(("point", (3.3 * np.cos(b), 3.3 * np.sin(b))))
        else:
            a = rng.uniform(0.0, 2.0 * np.pi)
            out.append(("plane", (np.cos(a), np.sin(a))))
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_solve_range_noalloc_matches_solve_range(fhw, precision):
    curves = [Wk.kite(), Wk.star_pool(1, 4)[0]]
    systems = [(0, 12.0, 160), (0, 13.5, 160), (1, 20.0, 224), (1, 21.0, 224), (0, 30.0, 352)]
    c = fhw.Context()
    try:
        say("noalloc vs solve_range", precision)
        c.plan_systems(curves, systems, precision=precision, refine_tol=1e-13, refine_max=10)
        c.factor()
        # call 1: every system, 11 incidences (two groups of the solve loop)
        # call 2: a smaller input, one system and 3 incidences
        for s0, count, inc in ((0, 5, _incidences(11, 1)), (3, 1, _incidences(3, 2))):
            ref, rres, rsw = c.solve_range(s0, count, inc)
            got, gres, gsw = c.solve_range(s0, count, inc, noalloc=True)
            torch.cuda.synchronize()
            say("range", s0, count, "incidences", len(inc), "max |diff|",
                float((got - ref).abs().max()), "resid max", float(np.max(gres)))
            assert got.shape == ref.shape
            assert torch.equal(got, ref)
            assert np.array_equal(gres, rres) and np.array_equal(gsw, rsw)
            if precision == "fp32_refine":
                assert np.all(gres <= 1e-13) and np.all(gsw >= 1)
            else:
                assert np.all(gres == -1.0) and np.all(gsw == 0)
        # beyond the fixed array: refused, and the context stays usable
        many = [("plane", (1.0, 0.0))] * (fhw_max_incidences(fhw) + 1)
        with pytest.raises(fhw.FhwError) as e:
            c.solve_range(0, 1, many, noalloc=True)
        assert e.value.code == fhw.FHW_E_INVALID
        ref, _, _ = c.solve_range(1, 1, _incidences(2, 4))
        got, _, _ = c.solve_range(1, 1, _incidences(2, 4), noalloc=True)
        assert torch.equal(got, ref)
    finally:
        c.close()


def fhw_max_incidences(fhw):
    """FHW_NOALLOC_MAX_PAIRS from the header: the largest n_inc for one system."""
    import os
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fhw.h")).read()
    return int(re.search(r"#define FHW_NOALLOC_MAX_PAIRS (\d+)", hdr).group(1))
