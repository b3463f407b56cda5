"""Writes the oracle's densities on seeded subsets of the two full-size
frequency-domain workloads that no test can re-solve on the CPU in its own
time, for the GPU parity tests:

  star_batch   64 seeded star curves x 256 frequencies on (0, 120], N from 17
               points per wavelength (64 .. 2048): every 16th system, systems
               s = 16 i + 15 (frequency indices 15, 31, .., 255 of every
               curve: both workspace chunks and the largest N = 2048)
  kite_chirp   kite, 512 frequencies on (0, 200], N from 10 points per
               wavelength (64 .. 2976): every 16th frequency, j = 15, 31, ..,
               511 (the largest N included)

Per sampled system: N, 64 densities psi[idx] at idx = round(linspace(0,
N - 1, 64)), max |psi|, ||psi||_2, the relative residual ||g - A psi|| /
||g||, and an estimate of the infinity-norm condition number of A (LAPACK
zgecon on A's LU factors) for the error bound of the FP32-LU + refinement
path.  The densities come from the oracle's assembly and LAPACK solve; the
condition estimate is LAPACK's.  Run from the repository root:

    python tests/golden/make_golden_subsets.py star_batch kite_chirp

(about 2 min on 8 cores).  Output: tests/golden/<name>_psi_sub16.npz."""
import os
import sys
import time
from multiprocessing import Pool

os.environ.setdefault("OMP_NUM_THREADS", "1")   # one BLAS thread per worker process
import numpy as np  # noqa: E402
from scipy import linalg  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O          # noqa: E402
import workloads as Wk      # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
N_SAMPLES = 64


def sample_index(N):
    return np.round(np.linspace(0, N - 1, N_SAMPLES)).astype(np.int64)


def _one(args):
    curve, N, kappa, eta, p = args
    gm = O.geometry(curve, int(N))
    A = O.assemble(gm, kappa, eta)
    g = O.rhs_plane_wave(gm, kappa, eta, p)
    psi, res = O.solve_density(A, g)
    lu, _ = linalg.lu_factor(A)
    rcond, info = linalg.lapack.zgecon(lu, np.max(np.sum(np.abs(A), axis=1)), norm="I")
    idx = sample_index(N)
    return (psi[idx], float(np.max(np.abs(psi))), float(np.linalg.norm(psi)), res,
            float(1.0 / rcond) if rcond > 0 else float("inf"))


def systems(name):
    """(curve, N, kappa, eta, direction) of every sampled system, and the
    system indices."""
    if name == "star_batch":
        sb = Wk.star_batch()
        _, kappa = O.frequency_grid(sb["W"], sb["F"])
        eta = O.coupling(kappa)
        out, ids = [], []
        for k, cv in enumerate(sb["curves"]):
            Ns = O.discretization_sizes(kappa, O.curve_length(cv), **sb["rule"])
            for j in range(15, sb["F"], 16):
                out.append((cv, int(Ns[j]), float(kappa[j]), float(eta[j]), sb["direction"]))
                ids.append(k * sb["F"] + j)
        return out, ids
    if name == "kite_chirp":
        wl = Wk.kite_chirp()
        _, kappa = O.frequency_grid(wl.W, wl.F)
        eta = O.coupling(kappa)
        Ns = O.discretization_sizes(kappa, O.curve_length(wl.curve), **wl.N)
        js = list(range(15, wl.F, 16))
        return [(wl.curve, int(Ns[j]), float(kappa[j]), float(eta[j]), wl.direction) for j in js], js
    raise KeyError(name)


def make(name, workers):
    t0 = time.perf_counter()
    work, ids = systems(name)
    # largest first, so that the pool's tail is short
    order = sorted(range(len(work)), key=lambda i: -work[i][1])
    with Pool(workers) as pool:
        res = pool.map(_one, [work[i] for i in order], chunksize=1)
    out = [None] * len(work)
    for i, r in zip(order, res):
        out[i] = r
    Ns = np.array([w[1] for w in work], dtype=np.int64)
    np.savez(os.path.join(HERE, f"{name}_psi_sub16.npz"),
             system=np.array(ids, dtype=np.int64), N=Ns,
             psi=np.stack([r[0] for r in out]), psi_max=np.array([r[1] for r in out]),
             psi_norm2=np.array([r[2] for r in out]), resid=np.array([r[3] for r in out]),
             cond_inf=np.array([r[4] for r in out]))
    print(name, len(work), "systems", "N", int(Ns.min()), "..", int(Ns.max()),
          "max resid %.2e" % max(r[3] for r in out), "cond_inf max %.1f" % max(r[4] for r in out),
          "%.0f s" % (time.perf_counter() - t0), flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:] or ["star_batch", "kite_chirp"]:
        make(nm, min(8, os.cpu_count() or 1))
