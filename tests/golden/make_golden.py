"""Writes the oracle's time samples for a full-size workload at a subset of
its observation points, for the full-size GPU parity tests:

  kite_n1024   solve-throughput workload: kite, N = 1024 at each of 1024
               frequencies on (0, 69], slow chirp to T = 1e4 (about 7 min)
  kite_chirp   kite, 512 frequencies on (0, 200] with 10 points per
               wavelength (N = 64 .. 2976), the paper's chirp to T = 1e4
               (about 10 min)

Calls only the oracle and the seeded workload generators.  Run from the
repository root:  python tests/golden/make_golden.py kite_n1024 kite_chirp
Output: tests/golden/<workload name>_u_sample.npy and .json."""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O          # noqa: E402
import workloads as Wk      # noqa: E402

OBS_IDX = [0, 64, 128, 192]   # points on the radius-3 ring: angles 0, pi/2, pi, 3 pi/2
WORKLOADS = {"kite_n1024": Wk.kite_n1024, "kite_chirp": Wk.kite_chirp}


def make(key):
    wl = WORKLOADS[key]()
    obs = wl.obs[OBS_IDX]
    t0 = time.perf_counter()
    out = O.run(wl.curve, wl.W, wl.F, wl.N, wl.direction, wl.signal, wl.H, wl.tau0, obs, wl.times,
                return_all=True)
    here = os.path.dirname(os.path.abspath(__file__))
    np.save(os.path.join(here, f"{wl.name}_u_sample.npy"), out["u"])
    meta = dict(workload=wl.name, obs_index=OBS_IDX, n_times=len(wl.times),
                max_abs_u=float(np.max(np.abs(out["u"]))), max_abs_im=float(out["im_max"]),
                max_residual=float(np.max(out["res"])), N_min=int(np.min(out["Ns"])), N_max=int(np.max(out["Ns"])),
                windows=[int(out["ks"][0]), int(out["ks"][-1])],
                n_windows=int(len(out["ks"])), seconds=round(time.perf_counter() - t0, 1))
    with open(os.path.join(here, f"{wl.name}_u_sample.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(meta), flush=True)


if __name__ == "__main__":
    for key in sys.argv[1:] or ["kite_n1024"]:
        make(key)
