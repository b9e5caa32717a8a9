"""The oracle built with the address and undefined-behaviour sanitizers (gcc, host code only):
the 64^2 wall workload for 50 steps, a 3D lattice with walls, a periodic lattice with the
-phi grad mu force and a run without hydrodynamics must finish without a sanitizer report (an
out-of-bounds access, a use after free, a leak or an undefined operation aborts the run), and
give the same observables as the ordinary build."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synthetic as S
from oracle import Oracle, make_params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("no gcc")
    d = tmp_path_factory.mktemp("san")
    exe = str(d / "check_main")
    flags = ["-O1", "-g", "-std=c11", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all"]
    r = subprocess.run(["gcc", *flags, "-o", exe, os.path.join(SRC, "check_main.c"),
                        os.path.join(SRC, "lam_oracle.c"), "-fopenmp", "-lm"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe, d


CASES = {
    "c1_64sq_50": (S.model_params("c1_64sq"), S.initial_phi("c1_64sq"), 50),
    "3d_walls": (S.model_params("c3_256cube_xi0.1", nx=12, ny=10, nz=14),
                 S.phi0((14, 10, 12), seed=3), 6),
    "periodic_phi_grad_mu": (S.model_params("c1_64sq", nx=20, ny=16, walls=0, force_form=1,
                                            T0=0.8, Tw=0.8), S.phi0((16, 20), seed=4), 10),
    "no_hydro": (S.model_params("paper_2d_nohydro", nx=24, ny=20), S.phi0((20, 24), seed=5,
                                                                          amplitude=0.01), 10),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_oracle_clean_under_sanitizers(checker, case):
    exe, d = checker
    p, phi0, steps = CASES[case]
    pf, ff = d / f"{case}.params", d / f"{case}.phi"
    pf.write_bytes(bytes(make_params(p)))
    ff.write_bytes(np.ascontiguousarray(phi0, dtype=np.float64).tobytes())
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, str(pf), str(ff), str(steps)], capture_output=True, text=True,
                       env=env, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr
    mass, phisum, umax, fe, step, nonfinite = r.stdout.split()
    ob = Oracle(p).init_fields(phi0).step(steps).observables()
    assert int(step) == steps and int(nonfinite) == ob["nonfinite"]
    for got, want in ((float(phisum), ob["phi_sum"]), (float(fe), ob["free_energy"]),
                      (float(umax), ob["max_u"])):
        assert got == pytest.approx(want, rel=1e-12, abs=1e-12)
    assert float(mass) == pytest.approx(ob["mass_dev"], abs=1e-10)
