"""Host-side checks of the C-ABI library that need no GPU: it loads, exports every symbol that
include/lam.h declares, and rejects invalid parameter sets with LAM_EINVAL / LAM_ESIZE."""
import ctypes as C
import os
import re

import pytest

import paper_1102_3094_amd as lam
import synthetic as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(lam.LIB_PATH):
        from paper_1102_3094_amd.build import build
        build()
    return lam.load()


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lam.h")).read()
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\*)\s+(lam_\w+)\s*\(", src, re.M)))


def test_exports_every_declared_symbol(L):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(lam.EXPORTS)


def test_struct_layout_matches_header():
    # offsets the C compiler gives the header's structs, compared with the ctypes mirror
    import subprocess
    import tempfile
    code = r'''
#include <stdio.h>
#include <stddef.h>
#include "lam.h"
int main(){printf("%zu %zu %zu %zu %zu\n", sizeof(lam_params), offsetof(lam_params, body_force),
offsetof(lam_params, n_phi_sub), sizeof(lam_obs), offsetof(lam_obs, step)); return 0;}
'''
    with tempfile.TemporaryDirectory() as d:
        open(os.path.join(d, "t.c"), "w").write(code)
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), "-o", os.path.join(d, "t"),
                        os.path.join(d, "t.c")], check=True)
        out = subprocess.run([os.path.join(d, "t")], capture_output=True, text=True).stdout.split()
    got = [C.sizeof(lam.lam_params), lam.lam_params.body_force.offset,
           lam.lam_params.n_phi_sub.offset, C.sizeof(lam.lam_obs), lam.lam_obs.step.offset]
    assert [int(v) for v in out] == got


@pytest.mark.parametrize("bad", [dict(tau=0.5), dict(b=0.0), dict(c=-1.0), dict(nx=4),
                                 dict(dim=4), dict(force_form=3), dict(pop_storage=2),
                                 dict(n_phi_sub=1), dict(n_T_sub=1, xi=1.0),
                                 dict(nx=32768, ny=32768),                 # N 4 B = 2^32
                                 dict(nx=65536, ny=32768, pop_storage=1),   # N 2 B = 2^32
                                 dict(dim=3, nx=1024, ny=1024, nz=1024)])   # N 4 B = 2^32
def test_invalid_parameters_rejected(L, bad):
    p = S.model_params("c1_64sq", **bad)
    with pytest.raises(lam.LamError) as e:
        lam.workspace_bytes(p)
    assert e.value.code == lam.LAM_EINVAL


def test_largest_2d_lattice_accepted(L):
    """Just below the 32-bit plane-offset limit of the D2Q9 step kernel (sizing only)."""
    assert lam.workspace_bytes(S.model_params("c1_64sq", nx=32768, ny=32767)) > 0


def test_unstable_override_allowed_when_forced(L):
    p = S.model_params("c1_64sq", n_phi_sub=1, allow_unstable=1)
    assert lam.workspace_bytes(p) > 0


def test_create_validates_workspace(L):
    p = lam.make_params(S.model_params("c1_64sq"))
    n = C.c_size_t()
    assert L.lam_workspace_bytes(C.byref(p), C.byref(n)) == 0
    h = C.c_void_p()
    # too small: rejected before any device access
    rc = L.lam_create(C.byref(p), C.c_void_p(1 << 20), n.value - 1, None, C.byref(h))
    assert rc == lam.LAM_ESIZE
    assert b"workspace" in L.lam_last_error(None)
    # misaligned
    rc = L.lam_create(C.byref(p), C.c_void_p((1 << 20) + 8), n.value + 64, None, C.byref(h))
    assert rc == lam.LAM_EINVAL


def test_substep_rule_host(L):
    """The library's automatic sub-step counts (host code, no GPU needed)."""
    for name, want in (("c1_64sq", 2), ("paper_2d_tau5", 1)):
        p = lam.make_params(S.model_params(name))
        n = C.c_size_t()
        assert L.lam_workspace_bytes(C.byref(p), C.byref(n)) == 0
        h = C.c_void_p()
        assert L.lam_create(C.byref(p), C.c_void_p(1 << 20), n.value, None, C.byref(h)) == 0
        a, b = C.c_int32(), C.c_int32()
        L.lam_substeps(h, C.byref(a), C.byref(b))
        L.lam_destroy(h)
        assert a.value == want and b.value == 1


def test_ensemble_validation(L):
    a = S.model_params("c1_64sq")
    b = S.model_params("c1_64sq", nx=100, tau=0.7)
    arr = (lam.lam_params * 2)(lam.make_params(a), lam.make_params(b))
    n = C.c_size_t()
    assert L.lam_ensemble_workspace_bytes(arr, 2, C.byref(n)) == 0 and n.value > 0
    c = S.model_params("c1_64sq", kappa=-0.03, c=0.03, T0=0.0075, Tw=0.0045, Tc=0.005)
    arr = (lam.lam_params * 2)(lam.make_params(a), lam.make_params(c))
    assert L.lam_ensemble_workspace_bytes(arr, 2, C.byref(n)) == lam.LAM_EINVAL
    assert b"sub-step" in L.lam_ensemble_last_error(None)
    d = S.model_params("c3_256cube_xi0.1", nx=16, ny=16, nz=16)
    arr = (lam.lam_params * 2)(lam.make_params(a), lam.make_params(d))
    assert L.lam_ensemble_workspace_bytes(arr, 2, C.byref(n)) == lam.LAM_EINVAL


@pytest.mark.parametrize("name,over", [("c1_64sq", dict()), ("c1_64sq", dict(pop_storage=1)),
                                       ("c1_64sq", dict(nx=72, ny=40)),
                                       ("c3_256cube_xi0.1", dict(nx=37, ny=12, nz=70)),
                                       ("c3_256cube_xi0.1", dict(nx=64, ny=16, nz=9, pop_storage=1))])
def test_guard_bands_separate_every_region(L, name, over):
    """Guard bands: one at the workspace start and one behind every region, each 256-byte aligned,
    none inside the room a region needs, the last one ending the workspace (host only)."""
    p = S.model_params(name, **over)
    offs = lam.guard_layout(p)
    total = lam.workspace_bytes(p)
    assert len(offs) == 14 and offs[0] == 0
    assert all(o % 256 == 0 for o in offs)
    assert offs[-1] + lam.LAM_GUARD_BYTES == total
    N = p["nx"] * p["ny"] * (p["nz"] if p["dim"] == 3 else 1)
    Q = 9 if p["dim"] == 2 else 19
    esz = 2 if p.get("pop_storage", 0) else 4
    nrows = p["ny"] if p["dim"] == 2 else p["nz"]
    need = [Q * N * esz] * 2 + [4 * N] * 4 + [4 * p["dim"] * N] + [4 * nrows] * 3
    for i, b in enumerate(need):  # region i lies between band i and band i + 1
        assert offs[i + 1] - (offs[i] + lam.LAM_GUARD_BYTES) >= b
    gaps = [offs[i + 1] - offs[i] - lam.LAM_GUARD_BYTES for i in range(13)]
    assert min(gaps) > 0
