"""GPU parity of the fitting step (Sec. 4.1, eq. (15)) and of pseudo-open-loop
control (Sec. 4.2, Alg. 4.1) against the FP64 oracle, through the C ABI."""
import numpy as np
import pytest

import oracle as O
import workloads as WL
from tests.gpu_common import record, rel, require_gpu, say, setup, to_dev, to_np
from workloads.fitting import fitting_directions, fitting_systems, mirror_wfs_system

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_fitting_e_elt(dt):
    require_gpu()
    import torch
    from paper_1302_3734_amd.fitting import Fitter
    cfg = WL.config_c2()
    atm, dm = fitting_systems(cfg)
    Sfa = O.System(atm, [1.0] * 25)
    Sfd = O.System(dm, [1.0] * 25)
    truth = WL.layer_screens(cfg, 0, seed_frame=0)
    a_ref = O.fit(Sfa, Sfd, truth, 4, J=Sfd.jacobi_separable())
    tdt = torch.float64 if dt == "f64" else torch.float32
    fitter = Fitter(atm, dm, dtype=dt)
    J = to_np(fitter.dm.precond_diag())
    assert np.max(np.abs(J - Sfd.jacobi_separable()) / J) < 1e-12
    lay = to_dev(np.concatenate([t.ravel() for t in truth])[None], tdt)
    a = torch.zeros(1, fitter.n_act, dtype=tdt, device="cuda")
    fitter.fit(lay, a, warm_start=False)
    e = rel(to_np(a).ravel(), a_ref)
    say(f"[fit-{dt}] e_a {e:.2e}")
    record("fit-E-ELT", dt, (e,) * 3, ((1e-11 if dt == "f64" else 1e-5),) * 3)
    assert e < (1e-11 if dt == "f64" else 1e-5)
    fitter.close()


def test_polc_closed_loop_steps():
    """Four control steps on the 8 m system with two mirrors, fed the same
    residual slopes: every command vector matches the oracle's loop to the
    FP64 bar (the oracle's own loop moves by ~6e-14 when its slopes change by
    one ulp)."""
    require_gpu()
    import torch
    from paper_1302_3734_amd.fitting import PolcController
    cfg = WL.config_c1()
    mir = [{"altitude": 0.0, "pitch": 0.5, "n": 20}, {"altitude": 4e3, "pitch": 1.0, "n": 12}]
    atm, dm = fitting_systems(cfg, mirrors=mir, directions=fitting_directions(1.0, 3), n_sub=16)
    dmw = mirror_wfs_system(cfg, mir)
    S, sig, s, _ = setup(cfg)
    Sa = O.System(dmw, sig)
    ora = O.Polc(S, Sa, O.System(atm, [1.0] * 9), O.System(dm, [1.0] * 9), gain=0.4,
                 n_iter=10, fit_iter=4)
    gpu = PolcController(cfg, sig, dmw, atm, dm, dtype="f64", gain=0.4, n_iter=10)
    for t in range(4):
        truth = WL.layer_screens(cfg, t, seed_frame=0)
        s_t = S.forward_layers(truth) - Sa.forward(ora.a_hist[0])
        a_o = ora.step(s_t)
        a_g = to_np(gpu.step(to_dev(s_t[None], torch.float64))).ravel()
        say(f"[polc] step {t}: e_a {rel(a_g, a_o):.2e}")
        record("POLC-C1", "f64", (rel(a_g, a_o),) * 3, (1e-11,) * 3)
        assert rel(a_g, a_o) < 1e-11, t
    gpu.close()
