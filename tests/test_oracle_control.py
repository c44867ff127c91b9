"""Pins of the oracle's fitting step (Sec. 4.1, eq. (15)) and pseudo-open-loop
control (Sec. 4.2, Alg. 4.1)."""
import numpy as np
import pytest

import oracle as O
import workloads as WL
from tests.dense import assemble
from tests.tiny import tiny_config
from workloads.fitting import fitting_directions, fitting_systems, mirror_wfs_system

MIRRORS = [{"altitude": 0.0, "pitch": 0.5, "n": 12}, {"altitude": 6e3, "pitch": 1.0, "n": 8}]


def _systems(alpha=1.0):
    cfg = tiny_config(tt=False)
    cfg["alpha"] = alpha
    atm, dm = fitting_systems(cfg, mirrors=MIRRORS, directions=fitting_directions(1.0, 3), n_sub=8)
    return cfg, atm, dm


def test_fitting_operator_matches_dense_assembly():
    cfg, atm, dm = _systems()
    A, _, S = assemble(dm, [1.0] * len(dm["wfs"]))
    v = np.random.default_rng(0).standard_normal(S.n)
    assert np.linalg.norm(S.apply_A(v) - A @ v) < 1e-12 * np.linalg.norm(A @ v)
    assert np.max(np.abs(A - A.T)) < 1e-12 * np.max(np.abs(A))
    Ap, _, _ = assemble(dm, [1.0] * len(dm["wfs"]), precond_only=True)
    assert np.max(np.abs(S.jacobi_separable() - np.diag(Ap)) / np.diag(Ap)) < 1e-12
    assert np.max(np.abs(S.jacobi_bruteforce() - np.diag(Ap)) / np.diag(Ap)) < 1e-12


def test_fitting_reproduces_a_mirror_wavefront():
    # a wavefront made by the mirrors themselves is fitted to the Tikhonov
    # floor: |H a - H a_true| / |H a_true| is tiny once CG has converged
    cfg, atm, dm = _systems()
    Sd = O.System(dm, [1.0] * len(dm["wfs"]))
    a_true = np.random.default_rng(1).standard_normal(Sd.n)
    target = Sd.forward(a_true)
    b = Sd.rhs(target)
    J = Sd.jacobi_separable()
    res = []
    for k in (2, 4, 8, 200):
        a, _ = O.pcg(Sd.apply_A, b, k, jacobi=J)
        res.append(np.linalg.norm(Sd.forward(a) - target) / np.linalg.norm(target))
    assert res[-1] < 1e-3 and res[0] > res[-1]


def test_polc_follows_the_delayed_integrator_recursion():
    # With R exact (converged inner solves) and a static atmosphere, s_ol is
    # the same every step, R s_ol = a*, and Alg. 4.1 reduces to
    # e_t = e_{t-1} - g e_{t-2} for e_t = a_t - a*.  A strong prior keeps the
    # inner tomography solves fully converged in a few hundred iterations.
    cfg, atm, dm = _systems(alpha=1000.0)
    S0 = O.System(cfg, [1.0] * len(cfg["wfs"]))
    scr = WL.layer_screens(cfg, 0)
    clean = S0.forward_layers(scr)
    sig = [0.05] * len(cfg["wfs"])
    St = O.System(cfg, sig)
    Sa = O.System(mirror_wfs_system(cfg, MIRRORS), sig)
    Sfa = O.System(atm, [1.0] * len(atm["wfs"]))
    Sfd = O.System(dm, [1.0] * len(dm["wfs"]))
    g = 0.4
    loop = O.Polc(St, Sa, Sfa, Sfd, gain=g, n_iter=400, fit_iter=300)
    c, _ = O.pcg(St.apply_A, St.rhs(clean), 400, jacobi=St.jacobi_separable())
    astar = O.fit(Sfa, Sfd, St.to_layers(c), 300, J=Sfd.jacobi_separable())
    e = [-astar, -astar]                               # a_{-2} = a_{-1} = 0
    for t in range(8):
        s = clean - Sa.forward(loop.a_hist[0])         # residual slopes for a_{t-2}
        a = loop.step(s)
        e.append(e[-1] - g * e[-2])
        assert np.linalg.norm((a - astar) - e[-1]) < 1e-6 * np.linalg.norm(astar), t


def test_pseudo_open_loop_slopes_do_not_depend_on_the_mirrors():
    # s_ol = (G P phi - A^ a) + A^ a: the open-loop slopes for any command
    cfg, atm, dm = _systems()
    sig = [0.05] * len(cfg["wfs"])
    St = O.System(cfg, sig)
    Sa = O.System(mirror_wfs_system(cfg, MIRRORS), sig)
    scr = WL.layer_screens(cfg, 0)
    clean = St.forward_layers(scr)
    a = np.random.default_rng(3).standard_normal(Sa.n)
    s_ol = (clean - Sa.forward(a)) + Sa.forward(a)
    assert np.allclose(s_ol, clean, rtol=0, atol=1e-12 * np.abs(clean).max())
