"""Autotuner of the LU panel kernel's tile shape (sub-panel width W and waves
per SIMD) per precision, workgroup size and rows per thread.

    python -m paper_1807_02718_amd.tune build [jobs] [families]   # CPU: variant libraries
    python -m paper_1807_02718_amd.tune measure [all|big|tall]     # GPU: time them
    python -m paper_1807_02718_amd.tune write [results.json]       # CPU: csrc/panel_table.h
(families: PB, PBT, 1024, comma-separated; big times the kite at N = 1024
with 1024 frequencies only, the shape of the PB cases; tall times star-curve
batches with panels of 1025-2048 rows (N = 1536) and 2049-4096 rows
(N = 4096), the PBT cases)
    python -m paper_1807_02718_amd.tune gemm-build | gemm-measure | gemm-write
        the same for the GEMM kernel (k_lu_gemm): K-chunk and workgroups per CU
        per precision, timed as the update + TRSM stages of the kite batch at
        N = 1024 (both precisions) and of 16 star curves x 256 frequencies
        (FP64), written to csrc/gemm_table.h

Each variant differs from the current table (csrc/panel_table.h) in one case,
set to one candidate whose registers fit without spilling (checked from the
compiler's resource report). `measure` times the panel stage of
fhw_solve_densities with the library's own HIP-event timers on the kite: for the
large-batch cases (batches above 256 matrices: workgroup size 256, 512 or 1024,
W and waves per SIMD) N = 1024 with 1024 frequencies, whose shrinking panels
pass through R = 4, 2 and 1 rows per 256 threads; for the 1024-thread cases
the sum of N = 1024 with 64 frequencies (R = 1) and N = 4096 with 16
frequencies (R = 4, 2, 1); for the tall panels of large batches (R = 8 and
16 rows per 256 threads: workgroup size, W and waves per SIMD) 512 systems at
N = 1536 and 300 at N = 4096 on four star curves, factored by fhw_factor.
`write` keeps, per case, the fastest variant if it beats the current table by
more than 1%.
"""
from __future__ import annotations

import json
import os
import re
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
TUNE = os.path.join(HERE, "_tune")
TABLE = os.path.join(CSRC, "panel_table.h")

# candidate values per case family; the spill check drops the rest.  1024:
# batches of at most 256 matrices, (W, waves per SIMD) at 1024 threads; PB:
# larger batches, (threads, W, waves per SIMD, columns in flight PD).  An
# earlier sweep of PB over 512 and 1024 threads and W = 4 and 16 found every
# such shape slower than 256 threads with W = 8 (profiles/), so this one
# varies the occupancy and the lazy loads in flight.
CANDIDATES = {
    1024: [(4, 4), (8, 4), (16, 4)],
    "PB": [(256, 8, e, d) for e in (4, 3, 2) for d in (0, 1, 2, 4, 8)],
    "PBT": [(256, 4, 2, 0), (256, 2, 2, 0), (256, 2, 1, 0), (512, 8, 4, 0), (512, 8, 2, 0), (512, 4, 4, 0),
            (512, 4, 2, 0), (1024, 8, 4, 0), (1024, 8, 2, 0), (1024, 4, 4, 0)],
}
CASES = ([(p, pt, r) for p in ("F32", "F64") for pt in ("PB", 1024) for r in (1, 2, 4)] +
         [(p, "PBT", r) for p in ("F32", "F64") for r in (8, 16)])


def case_name(p, pt, r):
    return f"FHW_PB_{p}_R{r}" if pt in ("PB", "PBT") else f"FHW_PT_{p}_{pt}_R{r}"


def read_table(path=TABLE):
    tab = {}
    for m in re.finditer(r"#define (FHW_P[TB]_\w+) (\d+(?:, \d+)+)", open(path).read()):
        tab[m.group(1)] = tuple(int(x) for x in m.group(2).split(", "))
    return tab


def write_table(tab, path=TABLE):
    src = open(TABLE).read()
    for name, vals in tab.items():
        src = re.sub(rf"#define {name} \d+(?:, \d+)+", f"#define {name} " + ", ".join(str(v) for v in vals), src)
    open(path, "w").write(src)


def variants(families=None):
    """name -> (table, changed case or None); families limits the swept cases."""
    base = read_table()
    out = {"base": (dict(base), None)}
    for p, pt, r in CASES:
        if families and str(pt) not in families:
            continue
        name = case_name(p, pt, r)
        for cand in CANDIDATES[pt]:
            if tuple(cand) == base[name] or (pt in ("PB", "PBT") and cand[0] > 256 * r):
                continue   # the current value, or more threads than panel rows
            t = dict(base)
            t[name] = tuple(cand)
            out[f"{name}_" + "_".join(str(v) for v in cand)] = (t, (p, pt, r))
    return out


def _spill_free(report, p, pt, r, *vals):
    """The panel instantiation of this case compiled without VGPR spills."""
    T = "f" if p == "F32" else "d"
    if pt in ("PB", "PBT"):
        threads, w, e, d = vals
        rows = (256 * r + threads - 1) // threads
        key = f"k_lu_panelI{T}Li{rows}ELi{w}ELi{e}ELi{threads}ELi{d}E"
    else:
        w, e = vals
        key = f"k_lu_panelI{T}Li{r}ELi{w}ELi{e}ELi{pt}ELi0E"
    blocks = report.split("Function Name: ")
    for b in blocks:
        if b.startswith("_Z10") and key in b.split()[0]:
            m = re.search(r"VGPRs Spill: (\d+)", b)
            return m is not None and int(m.group(1)) == 0
    return False


def build(jobs=4, families=None):
    from . import build as B
    B.build(jobs=jobs)   # the other objects, current table
    objs = [os.path.join(B.BUILD, s.replace(".hip", ".o")) for s in B.SOURCES if s != "lu.hip"]
    shutil.rmtree(TUNE, ignore_errors=True)
    os.makedirs(TUNE)
    vs = variants(families)

    def one(item):
        name, (tab, case) = item
        d = os.path.join(TUNE, name)
        os.makedirs(os.path.join(d, "paper_1807_02718_amd"))
        shutil.copy(os.path.join(CSRC, "lu.hip"), d)
        shutil.copy(TABLE, d)
        write_table(tab, os.path.join(d, "panel_table.h"))
        o = os.path.join(d, "lu.o")
        r = subprocess.run([B.HIPCC, *B.FLAGS, "-I", CSRC, "-c", os.path.join(d, "lu.hip"), "-o", o,
                            "-Rpass-analysis=kernel-resource-usage"], capture_output=True, text=True)
        if r.returncode:
            return name, False, r.stderr[-500:]
        ok = case is None or _spill_free(r.stderr, *case, *tab[case_name(*case)])
        if not ok:
            shutil.rmtree(d)
            return name, False, "spills"
        r = subprocess.run([B.HIPCC, "-shared", "-fPIC", f"--offload-arch={B.ARCH}", *objs, o, "-o",
                            os.path.join(d, "paper_1807_02718_amd", "libfhw.so")], capture_output=True, text=True)
        os.remove(o)
        for f in ("__init__.py", "fhw.py"):
            shutil.copy(os.path.join(HERE, f), os.path.join(d, "paper_1807_02718_amd", f))
        json.dump(tab, open(os.path.join(d, "table.json"), "w"))
        return name, r.returncode == 0, r.stderr[-300:]

    with ThreadPoolExecutor(jobs) as ex:
        for name, ok, msg in ex.map(one, vs.items()):
            print(f"{name}: {'ok' if ok else 'skipped (' + msg.strip()[:80] + ')'}", flush=True)


_TIMER = r"""
import json, sys, numpy as np
sys.path.insert(0, sys.argv[1]); sys.path.insert(1, sys.argv[2])
import torch
from paper_1807_02718_amd import fhw
import workloads as Wk
out = {}
shapes = ((1024, 1024), (64, 1024), (16, 4096)) if sys.argv[3] == "all" else ((1024, 1024),)
if sys.argv[3] == "tall":
    shapes = ()
    curves = Wk.star_pool(4, 0)
    for prec in ("fp32_refine", "fp64"):
        for N, n_sys in ((1536, 512), (4096, 300)):
            ctx = fhw.Context()
            ctx.plan_systems(curves, [(q % 4, 100.0 + 0.5 * q, N) for q in range(n_sys)], precision=prec)
            ctx.factor()
            ts = []
            for _ in range(3):
                ctx.profile(True)
                ctx.factor()
                ts.append(ctx.profile_read()["lu_panel"][0])
                ctx.profile(False)
            ctx.close()
            out[f"{prec}_tall{N}"] = float(np.median(ts))
for prec in ("fp32_refine", "fp64"):
    for F, N in shapes:
        wl = Wk.kite_n1024(F=F)
        ctx = fhw.Context()
        ctx.plan(wl.curve, wl.W, F, N=N, precision=prec, refine_tol=1e-12, refine_max=10, direction=wl.direction)
        psi = torch.empty(int(ctx.psi_off[-1]), dtype=torch.complex128, device="cuda")
        ctx.solve_densities(psi)
        ts = []
        for _ in range(3):
            ctx.profile(True)
            ctx.solve_densities(psi)
            ts.append(ctx.profile_read()["lu_panel"][0])
            ctx.profile(False)
        ctx.close()
        out[f"{prec}_{F}_{N}"] = float(np.median(ts))
print(json.dumps(out), flush=True)
"""


def measure(shapes="all"):
    """Time every built variant; shapes = "all" (the three kite shapes),
    "big" (N = 1024 at 1024 frequencies only: the large-batch cases) or
    "tall" (the star-curve batches at N = 1536 and 4096: the tall panels)."""
    root = os.path.dirname(HERE)
    res = {}
    for name in sorted(os.listdir(TUNE)):
        d = os.path.join(TUNE, name)
        if not os.path.isfile(os.path.join(d, "table.json")):
            continue
        r = subprocess.run([sys.executable, "-c", _TIMER, d, root, shapes], capture_output=True, text=True,
                           timeout=300)
        line = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
        if r.returncode or not line:
            print(f"{name}: failed ({r.stderr.strip()[-200:]})", flush=True)
            continue
        res[name] = {"table": json.load(open(os.path.join(d, "table.json"))), "ms": json.loads(line[-1])}
        print(name, res[name]["ms"], flush=True)
    json.dump(res, open(os.path.join(TUNE, "results.json"), "w"), indent=1)


def write(results=None):
    res = json.load(open(results or os.path.join(TUNE, "results.json")))
    base = res["base"]
    tab = {k: tuple(v) for k, v in base["table"].items()}
    for p, pt, r in CASES:
        name = case_name(p, pt, r)
        prec = "fp32_refine" if p == "F32" else "fp64"
        if pt == "PB":
            keys = [f"{prec}_1024_1024"]
        elif pt == "PBT":
            keys = [f"{prec}_tall1536" if r == 8 else f"{prec}_tall4096"]
        else:
            keys = [f"{prec}_64_1024", f"{prec}_16_4096"]
        if not all(k in base["ms"] for k in keys):
            continue   # not timed in this sweep

        def cost(v):
            return sum(v["ms"][k] for k in keys)

        best, best_ms = tab[name], cost(base)
        for vn, v in res.items():
            if vn.startswith(name + "_") and cost(v) < best_ms * 0.99:
                best, best_ms = tuple(v["table"][name]), cost(v)
        if best != tab[name]:
            print(f"{name}: {tab[name]} -> {best} ({cost(base):.3f} -> {best_ms:.3f} ms panel stage)")
        tab[name] = best
    write_table(tab)
    print("wrote", TABLE)


# ---------------------------------------------------------------------------
# GEMM tile: K-chunk GK and workgroups per CU of k_lu_gemm, per precision
# ---------------------------------------------------------------------------
GEMM_TABLE = os.path.join(CSRC, "gemm_table.h")
GEMM_TUNE = os.path.join(HERE, "_tune_gemm")
GEMM_CANDIDATES = {"F32": [(gk, occ) for gk in (8, 16, 32) for occ in (2, 3, 4, 5)],
                   "F64": [(gk, occ) for gk in (8, 16, 32) for occ in (1, 2, 3, 4)]}


def read_gemm_table(path=GEMM_TABLE):
    src = open(path).read()
    out = {}
    for p in ("F32", "F64"):
        gk = int(re.search(rf"#define FHW_GEMM_GK_{p} (\d+)", src).group(1))
        occ = int(re.search(rf"#define FHW_GEMM_OCC_{p} (\d+)", src).group(1))
        out[p] = (gk, occ)
    return out


def write_gemm_table(tab, path=GEMM_TABLE):
    src = open(GEMM_TABLE).read()
    for p, (gk, occ) in tab.items():
        src = re.sub(rf"#define FHW_GEMM_GK_{p} \d+", f"#define FHW_GEMM_GK_{p} {gk}", src)
        src = re.sub(rf"#define FHW_GEMM_OCC_{p} \d+", f"#define FHW_GEMM_OCC_{p} {occ}", src)
    open(path, "w").write(src)


def gemm_variants():
    base = read_gemm_table()
    out = {"base": (dict(base), None)}
    for p, cands in GEMM_CANDIDATES.items():
        for gk, occ in cands:
            if (gk, occ) == base[p]:
                continue
            t = dict(base)
            t[p] = (gk, occ)
            out[f"{p}_GK{gk}_OCC{occ}"] = (t, p)
    return out


def _gemm_spill_free(report, p):
    T = "f" if p == "F32" else "d"
    blocks = report.split("Function Name: ")
    seen = False
    for b in blocks:
        if b.startswith(f"_Z9k_lu_gemmI{T}"):
            seen = True
            m = re.search(r"VGPRs Spill: (\d+)", b)
            if m is None or int(m.group(1)) != 0:
                return False
    return seen


def gemm_build(jobs=4):
    from . import build as B
    B.build(jobs=jobs)
    objs = [os.path.join(B.BUILD, s.replace(".hip", ".o")) for s in B.SOURCES if s != "lu.hip"]
    shutil.rmtree(GEMM_TUNE, ignore_errors=True)
    os.makedirs(GEMM_TUNE)

    def one(item):
        name, (tab, p) = item
        d = os.path.join(GEMM_TUNE, name)
        os.makedirs(os.path.join(d, "paper_1807_02718_amd"))
        shutil.copy(os.path.join(CSRC, "lu.hip"), d)
        shutil.copy(TABLE, d)
        shutil.copy(GEMM_TABLE, d)
        write_gemm_table(tab, os.path.join(d, "gemm_table.h"))
        o = os.path.join(d, "lu.o")
        r = subprocess.run([B.HIPCC, *B.FLAGS, "-I", CSRC, "-c", os.path.join(d, "lu.hip"), "-o", o,
                            "-Rpass-analysis=kernel-resource-usage"], capture_output=True, text=True)
        if r.returncode:
            return name, False, r.stderr[-500:]
        if p is not None and not _gemm_spill_free(r.stderr, p):
            shutil.rmtree(d)
            return name, False, "spills"
        r = subprocess.run([B.HIPCC, "-shared", "-fPIC", f"--offload-arch={B.ARCH}", *objs, o, "-o",
                            os.path.join(d, "paper_1807_02718_amd", "libfhw.so")], capture_output=True, text=True)
        os.remove(o)
        for f in ("__init__.py", "fhw.py"):
            shutil.copy(os.path.join(HERE, f), os.path.join(d, "paper_1807_02718_amd", f))
        json.dump(tab, open(os.path.join(d, "table.json"), "w"))
        return name, r.returncode == 0, r.stderr[-300:]

    with ThreadPoolExecutor(jobs) as ex:
        for name, ok, msg in ex.map(one, gemm_variants().items()):
            print(f"{name}: {'ok' if ok else 'skipped (' + msg.strip()[:80] + ')'}", flush=True)


_GEMM_TIMER = r"""
import json, sys, numpy as np
sys.path.insert(0, sys.argv[1]); sys.path.insert(1, sys.argv[2])
import torch
from paper_1807_02718_amd import fhw
import workloads as Wk
out = {}
wl = Wk.kite_n1024()
for prec in ("fp32_refine", "fp64"):
    ctx = fhw.Context()
    ctx.plan(wl.curve, wl.W, wl.F, N=wl.N, precision=prec, refine_tol=1e-12, refine_max=10, direction=wl.direction)
    psi = torch.empty(int(ctx.psi_off[-1]), dtype=torch.complex128, device="cuda")
    ctx.solve_densities(psi)
    ts = []
    for _ in range(3):
        ctx.profile(True)
        ctx.solve_densities(psi)
        pr = ctx.profile_read()
        ts.append(pr["lu_update"][0] + pr["lu_trsm"][0])
        ctx.profile(False)
    ctx.close()
    out["kite_" + prec] = float(np.median(ts))
sb = Wk.star_batch(n_curves=16)
ctx = fhw.Context()
ctx.plan(sb["curves"], sb["W"], sb["F"], precision="fp64", direction=sb["direction"], **sb["rule"])
psi = torch.empty(int(ctx.psi_off[-1]), dtype=torch.complex128, device="cuda")
ctx.solve_densities(psi)
ts = []
for _ in range(2):
    ctx.profile(True)
    ctx.solve_densities(psi)
    pr = ctx.profile_read()
    ts.append(pr["lu_update"][0] + pr["lu_trsm"][0])
    ctx.profile(False)
ctx.close()
out["stars16_fp64"] = float(np.median(ts))
print(json.dumps(out), flush=True)
"""


def gemm_measure():
    root = os.path.dirname(HERE)
    res = {}
    for name in sorted(os.listdir(GEMM_TUNE)):
        d = os.path.join(GEMM_TUNE, name)
        if not os.path.isfile(os.path.join(d, "table.json")):
            continue
        print("measuring", name, flush=True)
        r = subprocess.run([sys.executable, "-c", _GEMM_TIMER, d, root], capture_output=True, text=True,
                           timeout=300)
        line = [ln for ln in r.stdout.splitlines() if ln.startswith("{")]
        if r.returncode or not line:
            print(f"{name}: failed ({r.stderr.strip()[-200:]})", flush=True)
            continue
        res[name] = {"table": json.load(open(os.path.join(d, "table.json"))), "ms": json.loads(line[-1])}
        print(name, res[name]["ms"], flush=True)
    json.dump(res, open(os.path.join(GEMM_TUNE, "results.json"), "w"), indent=1)


def gemm_write(results=None):
    res = json.load(open(results or os.path.join(GEMM_TUNE, "results.json")))
    base = res["base"]
    tab = {k: tuple(v) for k, v in base["table"].items()}
    for p in ("F32", "F64"):
        keys = ["kite_fp32_refine"] if p == "F32" else ["kite_fp64", "stars16_fp64"]

        def cost(v):
            return sum(v["ms"][k] for k in keys)

        best, best_ms = tab[p], cost(base)
        for vn, v in res.items():
            if vn.startswith(p + "_GK") and cost(v) < best_ms * 0.99:
                best, best_ms = tuple(v["table"][p]), cost(v)
        if best != tab[p]:
            print(f"{p}: {tab[p]} -> {best} ({cost(base):.3f} -> {best_ms:.3f} ms update + TRSM)")
        tab[p] = best
    write_gemm_table(tab)
    print("wrote", GEMM_TABLE)


if __name__ == "__main__":
    cmd = sys.argv[1] if len(sys.argv) > 1 else ""
    if cmd == "build":
        build(int(sys.argv[2]) if len(sys.argv) > 2 else 4, sys.argv[3].split(",") if len(sys.argv) > 3 else None)
    elif cmd == "measure":
        measure(sys.argv[2] if len(sys.argv) > 2 else "all")
    elif cmd == "write":
        write(sys.argv[2] if len(sys.argv) > 2 else None)
    elif cmd == "gemm-build":
        gemm_build(int(sys.argv[2]) if len(sys.argv) > 2 else 4)
    elif cmd == "gemm-measure":
        gemm_measure()
    elif cmd == "gemm-write":
        gemm_write(sys.argv[2] if len(sys.argv) > 2 else None)
    else:
        print(__doc__)
        sys.exit(2)
