"""ORACLE (test infrastructure only): the fitting step and pseudo-open-loop
control in plain FP64 NumPy.

Fitting (Sec. 4.1, eq. (15)): mirror commands a minimising |H a - P phi| over
the fitting directions, as the normal equations (H^T H + alpha I) a = H^T P phi
solved by CG with a fixed iteration count (4 in the paper, Sec. 5.2).  H and P
are Systems whose sensors measure the phase at the pupil nodes; H's layers are
the mirror actuator grids (no wavelet transform).

Pseudo-open-loop control with a two-step delay (Sec. 4.2, Alg. 4.1):
    s_ol = s + A^ a_{t-2};  da = R s_ol - a_{t-2};  a_t = a_{t-1} + g da,
R = tomography (warm-started PCG, Sec. 5.1), W^-1, fitting.
"""
import numpy as np

from .pcg import pcg


def fit(S_atm, S_dm, layers, n_iter, a0=None, J=None):
    target = S_atm.forward_layers(layers)
    b = S_dm.rhs(target)
    a, _ = pcg(S_dm.apply_A, b, n_iter, x0=a0, jacobi=J)
    return a


class Polc:
    def __init__(self, S_tomo, S_ahat, S_fit_atm, S_fit_dm, gain, n_iter, fit_iter):
        self.St, self.Sa, self.Sfa, self.Sfd = S_tomo, S_ahat, S_fit_atm, S_fit_dm
        self.gain, self.n_iter, self.fit_iter = gain, n_iter, fit_iter
        self.Jt = S_tomo.jacobi_separable()
        self.Jf = S_fit_dm.jacobi_separable()
        self.c = np.zeros(S_tomo.n)
        self.a_fit = np.zeros(S_fit_dm.n)
        self.a_hist = [np.zeros(S_fit_dm.n), np.zeros(S_fit_dm.n)]
        self.steps = 0

    def mirror_slopes(self, a):
        return self.Sa.forward(a)

    def step(self, s):
        a2, a1 = self.a_hist
        s_ol = s + self.mirror_slopes(a2)
        warm = self.steps > 0
        self.c, _ = pcg(self.St.apply_A, self.St.rhs(s_ol), self.n_iter,
                        x0=self.c if warm else None, jacobi=self.Jt)
        layers = self.St.to_layers(self.c)
        self.a_fit = fit(self.Sfa, self.Sfd, layers, self.fit_iter,
                         a0=self.a_fit if warm else None, J=self.Jf)
        da = self.a_fit - a2
        a_new = a1 + self.gain * da
        self.a_hist = [a1, a_new]
        self.steps += 1
        return a_new
