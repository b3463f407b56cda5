"""The C-ABI library loads and exports every entry point include/fhw.h declares,
and the ctypes structs match the header's layout.  CPU only (no compute calls)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fhw.h")
LIB = os.path.join(ROOT, "paper_1807_02718_amd", "libfhw.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fhw_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_hot_path():
    names = declared_functions()
    for n in ("fhw_create", "fhw_destroy", "fhw_plan", "fhw_solve_densities", "fhw_eval_field", "fhw_synthesize",
              "fhw_assemble", "fhw_lu_factor", "fhw_lu_solve", "fhw_window_spectra", "fhw_fourier_coefficients",
              "fhw_geometry", "fhw_kress_weights"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfhw.so not built")
def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfhw.so not built")
def test_binding_loads_and_covers_the_abi():
    from paper_1807_02718_amd import fhw
    assert sorted(fhw.EXPORTED) == declared_functions()
    assert fhw.fhw_version() == 1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libfhw.so not built")
def test_struct_layouts(tmp_path):
    """ctypes layouts equal what the C compiler makes of include/fhw.h."""
    import subprocess
    from paper_1807_02718_amd import fhw
    structs = {"fhw_curve": fhw.fhw_curve, "fhw_problem": fhw.fhw_problem, "fhw_signal": fhw.fhw_signal,
               "fhw_windows": fhw.fhw_windows, "fhw_incidence": fhw.fhw_incidence, "fhw_system": fhw.fhw_system}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void){"]
    for sname, cls in structs.items():
        lines.append(f'printf("{sname} size %zu\\n", sizeof({sname}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{sname} {fname} %zu\\n", offsetof({sname}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    for line in filter(None, out):
        sname, field, val = line.split()
        cls = structs[sname]
        got = C.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(val), line


def test_oracle_is_not_imported_by_the_product():
    pkg = os.path.join(ROOT, "paper_1807_02718_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "from oracle" not in txt, f


def test_bessel_tables_are_current():
    """The generated table header matches what its generator writes now."""
    import subprocess
    import sys
    import tempfile
    csrc = os.path.join(ROOT, "paper_1807_02718_amd", "csrc")
    with tempfile.TemporaryDirectory() as d:
        src = open(os.path.join(csrc, "gen_bessel_tables.py")).read()
        gen = os.path.join(d, "gen_bessel_tables.py")
        open(gen, "w").write(src)
        # --check: a float64 emulation of the device's evaluation with these
        # tables stays within 5e-15 of mpmath's J0, Y0, J1, Y1 on (1e-5, 3e3)
        subprocess.run([sys.executable, gen, "--check"], check=True, cwd=d)
        assert open(os.path.join(d, "bessel_tables.h")).read() == open(os.path.join(csrc, "bessel_tables.h")).read()


def test_hankel_phase_sincos_emulated():
    """fhw_sincos_shift (sin and cos of z - pi/4 for the Hankel phase): its
    constants are pi/4 split in two rounded doubles, 2/pi rounded and the
    rounded Taylor coefficients 1/n!, and its steps, replayed here with
    correctly rounded fused multiply-adds, stay within 2.5e-16 of mpmath on
    3 <= z <= 1e7 (near multiples of pi/4 included)."""
    from fractions import Fraction
    import mpmath as mp
    mp.mp.prec = 200
    src = open(os.path.join(ROOT, "paper_1807_02718_amd", "csrc", "fhw_device.h")).read()
    body = src[src.index("void fhw_sincos_shift"):]
    body = body[:body.index("\n}\n")]
    hexf = lambda t: float.fromhex(t)
    hi = hexf(re.search(r"#define FHW_PIO4_HI (\S+)", src).group(1))
    lo = hexf(re.search(r"#define FHW_PIO4_LO (\S+)", src).group(1))
    tpi = hexf(re.search(r"#define FHW_2_OVER_PI (\S+)", src).group(1))
    assert hi == float(mp.pi / 4) and lo == float(mp.pi / 4 - mp.mpf(hi)) and tpi == float(2 / mp.pi)
    coef = [hexf(t) for t in re.findall(r"(-?0x1\.[0-9a-f]+p-?\d+)", body)]
    ps, pc = coef[:8], coef[8:]
    assert ps == [(-1) ** k * float(1 / mp.factorial(2 * k + 1)) for k in range(8, 0, -1)]
    assert pc == [(-1) ** k * float(1 / mp.factorial(2 * k)) for k in range(8, 1, -1)]

    def fma(a, b, c):
        return float(Fraction(a) * Fraction(b) + Fraction(c))

    def dev(z):
        k = float(round(fma(z, tpi, -0.5)))
        m = fma(2.0, k, 1.0)
        r = fma(-m, lo, fma(-m, hi, z))
        x = r * r
        s_ = ps[0]
        for c in ps[1:]:
            s_ = fma(s_, x, c)
        c_ = pc[0]
        for c in pc[1:]:
            c_ = fma(c_, x, c)
        sr = fma(r * x, s_, r)
        cr = fma(x * x, c_, fma(-0.5, x, 1.0))
        q = int(k)
        a, b = (cr, -sr) if q & 1 else (sr, cr)
        return (-a, -b) if q & 2 else (a, b)

    rng = np.random.default_rng(5)
    zs = list(np.geomspace(3.0, 1e7, 700)) + list(rng.uniform(3.0, 700.0, 300))
    zs += [float(mp.pi / 4 * n) for n in (5, 6, 7, 101, 4097, 123457)]
    zs += [np.nextafter(float(mp.pi / 4 * n), 0.0) for n in (8, 9, 1001)]
    worst = 0.0
    for z in zs:
        s_, c_ = dev(float(z))
        w = mp.mpf(float(z)) - mp.pi / 4
        worst = max(worst, abs(s_ - float(mp.sin(w))), abs(c_ - float(mp.cos(w))))
    assert worst < 2.5e-16, worst


def test_panel_table_round_trip(tmp_path):
    """The autotuner's table: every case the panel launcher reads is defined,
    a rewrite changes only the case asked for, and each variant differs from
    the table in exactly one case."""
    from paper_1807_02718_amd import tune
    tab = tune.read_table()
    assert set(tab) == {tune.case_name(*c) for c in tune.CASES}
    lu = open(os.path.join(tune.CSRC, "lu.hip")).read()
    for name in tab:
        assert name in lu
    name = tune.case_name("F64", 1024, 2)
    out = tmp_path / "panel_table.h"
    tune.write_table({name: (16, 1)}, str(out))
    back = tune.read_table(str(out))
    assert back[name] == (16, 1) and all(back[k] == v for k, v in tab.items() if k != name)
    for vname, (vt, case) in tune.variants().items():
        diff = [k for k in vt if vt[k] != tab[k]]
        assert (case is None and not diff) or diff == [tune.case_name(*case)], vname


def test_fc_tables_are_current():
    """The committed FC(Gram) continuation tables match what their generator
    writes now (60-digit least squares; about half a minute)."""
    import subprocess
    import sys
    import tempfile
    csrc = os.path.join(ROOT, "paper_1807_02718_amd", "csrc")
    with tempfile.TemporaryDirectory() as d:
        gen = os.path.join(d, "gen_fc_tables.py")
        open(gen, "w").write(open(os.path.join(csrc, "gen_fc_tables.py")).read())
        subprocess.run([sys.executable, gen], check=True, cwd=d)
        assert open(os.path.join(d, "fc_tables.h")).read() == open(os.path.join(csrc, "fc_tables.h")).read()
