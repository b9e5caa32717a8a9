"""Guard bands of the workspace (race and bounds check): after many steps, observables, S(k) and
the orientation histogram on ragged lattices in 2D and 3D, FP32 and FP16 populations, and on
ensemble members, every band still holds its pattern; a band damaged from the host is found and
named; initialising the fields again restores the bands."""
import numpy as np
import pytest

import synthetic as S

pytestmark = pytest.mark.gpu


CASES = [("c1_64sq", dict(nx=72, ny=40, Tw=0.9), 2),
         ("c1_64sq", dict(nx=130, ny=66, Tw=0.9, pop_storage=1), 2),
         ("c1_64sq", dict(nx=48, ny=96, Tw=0.9, walls=0, force_form=1), 2),
         ("c3_256cube_xi0.1", dict(nx=37, ny=12, nz=70, Tw=0.9), 3),
         ("c3_256cube_xi0.1", dict(nx=70, ny=9, nz=20, Tw=0.9, pop_storage=1), 3)]


@pytest.mark.parametrize("name,over,dim", CASES)
def test_guards_intact_after_steps(gpu, name, over, dim):
    import torch
    p = S.model_params(name, **over)
    shape = (p["ny"], p["nx"]) if dim == 2 else (p["nz"], p["ny"], p["nx"])
    sim = gpu.Sim(p).init_fields(torch.tensor(S.phi0(shape, seed=3), dtype=torch.float32))
    sim.check_guards()
    for _ in range(3):
        sim.step(37)
        sim.observables()
        sim.orientation(18)
        if dim == 2:
            sim.structure_factor(min(p["nx"], p["ny"]) // 2)
    sim.check_guards()


def test_guards_of_ensemble_members(gpu):
    members = [S.model_params("c1_64sq", nx=nx, ny=ny, Tw=0.9, pop_storage=ps)
               for nx, ny, ps in [(64, 64, 1), (40, 100, 1), (130, 72, 1)]]
    phis = [S.phi0((m["ny"], m["nx"]), seed=20 + i) for i, m in enumerate(members)]
    ens = gpu.Ensemble(members).init_fields(phis).step(41)
    ens.synchronize()
    for view in ens.sims:
        view.check_guards()


def test_damaged_band_is_found_and_named(gpu):
    import torch
    p = S.model_params("c1_64sq", Tw=0.9)
    offs = gpu.guard_layout(p)
    sim = gpu.Sim(p)
    with pytest.raises(gpu.LamError) as e:
        sim.check_guards()  # fields not initialised: no bands yet
    assert e.value.code == gpu.LAM_EINVAL
    phi0 = torch.tensor(S.phi0((64, 64), seed=4), dtype=torch.float32)
    sim.init_fields(phi0).step(5)
    sim.check_guards()
    ws = sim.workspace  # the caller's workspace (uint8 device tensor)
    ws[offs[3] + 100] = 0x55  # band 3 follows phi[0]
    torch.cuda.synchronize()
    with pytest.raises(gpu.LamError) as e:
        sim.check_guards()
    assert e.value.code == gpu.LAM_ECORRUPT and "phi[0]" in str(e.value)
    sim.init_fields(phi0)  # refills the bands
    sim.check_guards()
    assert np.isfinite(sim.observables()["mass_dev"])
