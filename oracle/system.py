"""ORACLE (test infrastructure only): the wavelet-domain MAP normal equations of
the MCAO tomography problem, matrix-free, in plain FP64 NumPy.

System (Sec. 5.1, eq. (19)):
    (A~^T C^-1 A~ + alpha D) c = A~^T C^-1 s,   A~_m = Gamma_m P_m W^-1,
with the operator written per guide star as in Sec. 5.1: laser guide stars use
C^_m^-1 = (I - T) C~_m^-1 (I - T) (Sec. 4.3, eqs. (17)-(18)), natural guide stars
use C~_m^-1.  The noise covariance is block diagonal with one 2x2 block per
subaperture (Sec. 4.3, eq. (16)); sigma^2 I by default.

The prior D is diagonal in the wavelet basis (Sec. 3, eq. (13) and the D_l
display before it): D = (K_out^(-11/3) + 2^((11/3) j)) / c_rho(h).  Readings
used here: K_out is the outer-scale length L0; the scale term 2^j is the
spatial frequency nu_k = 2^-k / d of a level-k coefficient (k = 1 finest; the
final low-pass band takes k = J); the discrete coefficients carry a factor d^2;
c_rho(h) = 0.023 w_l r0^(-5/3).

The modified Jacobi preconditioner (Sec. 5.1, display for J) is the diagonal of
the sum over the preconditioner's sensors of A~_m^T C~_m^-1 A~_m (C~, not C^)
plus alpha D.  It is computed here in two independent ways: by brute force,
one basis vector at a time, and by the separable closed form that follows
from the tensor-product structure of the 2-D basis and of the bilinear
projection.

Coefficient vectors: per layer an N x N row-major Mallat array, layers
concatenated.  Slope vectors: per sensor, x-slopes of the active
subapertures (or active low-order cells) in row-major order, then y-slopes.

The fitting step (Sec. 4.1, eq. (15)) reuses this system: its unknowns are the
actuator grids of the deformable mirrors (piecewise bilinear surfaces, treated
as "layers" at the mirror altitudes, with no wavelet transform: levels = 0),
its sensors measure the phase itself at the pupil nodes in each fitting
direction ("kind": "phase", one value per node that is a corner of an active
subaperture, weight 1), and its regulariser is alpha times the identity, a
small Tikhonov term that selects the minimum-norm least-squares solution.
"""
import math

import numpy as np

from . import geometry as geo
from . import wavelet as wav


class System:
    def __init__(self, cfg, sigmas, cinv_blocks=None, h=None):
        self.cfg = cfg
        self.levels = int(cfg["levels"])
        self.h = wav.db3_lowpass() if h is None else np.asarray(h, dtype=np.float64)
        self.alpha = float(cfg["alpha"])
        self.layers = cfg["layers"]
        self.N = [int(L["n"]) for L in self.layers]
        self.layer_off = np.concatenate([[0], np.cumsum([n * n for n in self.N])]).astype(int)
        self.n = int(self.layer_off[-1])
        D = float(cfg["diameter"])
        self.sensors = []
        for m, w in enumerate(cfg["wfs"]):
            n_sub = int(w["n_sub"])
            mask = geo.subaperture_mask(n_sub, D, float(cfg["obstruction"]))
            xn = geo.node_coords(n_sub, D)
            axes = []
            for L in self.layers:
                hl = float(L["altitude"])
                s = 1.0 - hl / float(w["H"]) if w["lgs"] else 1.0
                ix0, tx = geo.bilinear_axis(xn, s, w["theta"][0] * hl, L["n"], L["spacing"])
                jy0, ty = geo.bilinear_axis(xn, s, w["theta"][1] * hl, L["n"], L["spacing"])
                axes.append((s, ix0, tx, jy0, ty))
            phase = w.get("kind", "sh") == "phase"
            k = int(w["tt_aggregate"])
            cells = geo.aggregation_cells(mask, k) if k else None
            node_mask = None
            if phase:
                node_mask = np.zeros((n_sub + 1, n_sub + 1), dtype=bool)
                for di in (0, 1):
                    for dj in (0, 1):
                        node_mask[di:di + n_sub, dj:dj + n_sub] |= mask
                S = int(node_mask.sum())
            else:
                S = len(cells) if cells is not None else int(mask.sum())
            if cinv_blocks is not None and cinv_blocks[m] is not None:
                blk = np.asarray(cinv_blocks[m], dtype=np.float64).reshape(S, 3)
            else:
                sg = float(sigmas[m])
                blk = np.tile([sg ** -2, 0.0, sg ** -2], (S, 1))
            self.sensors.append({
                "lgs": bool(w["lgs"]), "n_sub": n_sub, "mask": mask, "nodes": xn, "axes": axes,
                "cells": cells, "S": S, "blocks": blk, "phase": phase, "node_mask": node_mask,
                "nmeas": S if phase else 2 * S,
                "remove_tt": bool(w["remove_tt"]) and not phase,
                "in_precond": bool(w["in_precond"]),
                "theta": w["theta"], "H": float(w["H"]),
            })
        self.slope_off = np.concatenate(
            [[0], np.cumsum([s["nmeas"] for s in self.sensors])]).astype(int)
        self.n_slopes = int(self.slope_off[-1])
        self.D = self.prior_diag()

    # ---- coefficient <-> layer -------------------------------------------------
    def split(self, c):
        return [np.asarray(c[self.layer_off[l]:self.layer_off[l + 1]], dtype=np.float64)
                .reshape(N, N) for l, N in enumerate(self.N)]

    def join(self, arrs):
        return np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in arrs])

    def to_layers(self, c):
        """W^-1: coefficients -> layer fields (list of N x N arrays)."""
        return [wav.idwt2(cl, self.levels, self.h) for cl in self.split(c)]

    def to_coeffs(self, layers):
        """W: layer fields -> coefficient vector."""
        return self.join([wav.fdwt2(p, self.levels, self.h) for p in layers])

    # ---- one sensor ------------------------------------------------------------
    def _project(self, sen, layers):
        """P_m: sum over layers of bilinear samples at the sensor's nodes."""
        u = 0.0
        for (s, ix0, tx, jy0, ty), phi in zip(sen["axes"], layers):
            u = u + geo.project_layer(phi, ix0, tx, jy0, ty)
        return u

    def _project_adjoint(self, sen, v):
        return [geo.project_layer_adjoint(v, ix0, tx, jy0, ty, N)
                for (s, ix0, tx, jy0, ty), N in zip(sen["axes"], self.N)]

    def _measure(self, sen, u):
        """Gamma_m: Fried slopes, aggregated into low-order cells if asked; a
        phase sensor returns the phase at its pupil nodes."""
        if sen["phase"]:
            return u[sen["node_mask"]]
        fine = geo.fried_slopes(u, sen["mask"])
        if sen["cells"] is None:
            return fine
        mask = sen["mask"]
        Sf = int(mask.sum())
        sx = np.zeros(mask.shape)
        sy = np.zeros(mask.shape)
        sx[mask] = fine[:Sf]
        sy[mask] = fine[Sf:]
        ax = [sx[c].sum() / c.sum() for c in sen["cells"]]
        ay = [sy[c].sum() / c.sum() for c in sen["cells"]]
        return np.array(ax + ay)

    def _measure_adjoint(self, sen, w):
        if sen["phase"]:
            v = np.zeros(sen["node_mask"].shape)
            v[sen["node_mask"]] = w
            return v
        mask = sen["mask"]
        if sen["cells"] is not None:
            S = sen["S"]
            wx = np.zeros(mask.shape)
            wy = np.zeros(mask.shape)
            for q, c in enumerate(sen["cells"]):
                wx[c] += w[q] / c.sum()
                wy[c] += w[S + q] / c.sum()
            w = np.concatenate([wx[mask], wy[mask]])
        return geo.fried_adjoint(w, mask)

    @staticmethod
    def _tt_remove(s, S):
        """(I - T): remove the mean x-slope and the mean y-slope (the orthogonal
        projection onto tip and tilt of Sec. 4.3, eq. (17))."""
        out = s.copy()
        out[:S] -= s[:S].mean()
        out[S:] -= s[S:].mean()
        return out

    def _cinv(self, sen, s):
        """C~_m^-1 with one symmetric 2x2 block (a, b, c) per subaperture; a
        phase sensor weights each node by a."""
        if sen["phase"]:
            return sen["blocks"][:, 0] * s
        S = sen["S"]
        a, b, c = sen["blocks"][:, 0], sen["blocks"][:, 1], sen["blocks"][:, 2]
        return np.concatenate([a * s[:S] + b * s[S:], b * s[:S] + c * s[S:]])

    def _noise_weight(self, sen, s):
        """C^_m^-1 = (I-T) C~_m^-1 (I-T) for tip/tilt-removed laser guide
        stars (eq. (18)), else C~_m^-1."""
        if sen["remove_tt"]:
            return self._tt_remove(self._cinv(sen, self._tt_remove(s, sen["S"])), sen["S"])
        return self._cinv(sen, s)

    # ---- whole system ----------------------------------------------------------
    def forward_layers(self, layers):
        """s = A phi (eq. (6)): slopes of every sensor from layer fields."""
        return np.concatenate([self._measure(sen, self._project(sen, layers))
                               for sen in self.sensors])

    def forward(self, c):
        return self.forward_layers(self.to_layers(c))

    def slopes_of(self, s, m):
        return s[self.slope_off[m]:self.slope_off[m + 1]]

    def weight(self, s):
        return np.concatenate([self._noise_weight(sen, self.slopes_of(s, m))
                               for m, sen in enumerate(self.sensors)])

    def adjoint_layers(self, w):
        """sum_m P_m^T Gamma_m^T w_m: weighted slopes -> layer fields."""
        acc = [np.zeros((N, N)) for N in self.N]
        for m, sen in enumerate(self.sensors):
            v = self._measure_adjoint(sen, self.slopes_of(w, m))
            for l, g in enumerate(self._project_adjoint(sen, v)):
                acc[l] += g
        return acc

    def rhs(self, s):
        """b = W sum_m P_m^T Gamma_m^T C_m^-1 s_m (right side of eq. (19))."""
        return self.to_coeffs(self.adjoint_layers(self.weight(s)))

    def apply_A(self, c):
        """A c = W sum_m P_m^T Gamma_m^T C_m^-1 Gamma_m P_m W^-1 c + alpha D c."""
        data = self.to_coeffs(self.adjoint_layers(self.weight(self.forward(c))))
        return data + self.alpha * self.D * c

    def data_term(self, c):
        return self.to_coeffs(self.adjoint_layers(self.weight(self.forward(c))))

    # ---- prior and preconditioner --------------------------------------------
    def prior_level_values(self, l):
        """D of layer l for scale index k = 1..J (entry k-1); without a
        wavelet transform (levels = 0) the regulariser is the identity."""
        if self.levels == 0:
            return np.array([1.0])
        L = self.layers[l]
        d = float(L["spacing"])
        c_rho = 0.023 * float(L["weight"]) * float(self.cfg["r0"]) ** (-5.0 / 3.0)
        L0 = float(self.cfg["L0"])
        out = []
        for k in range(1, self.levels + 1):
            nu = 2.0 ** (-k) / d
            out.append(d * d * (L0 ** (-11.0 / 3.0) + nu ** (11.0 / 3.0)) / c_rho)
        return np.array(out)

    def prior_diag(self):
        parts = []
        for l, N in enumerate(self.N):
            vals = self.prior_level_values(l)
            if self.levels == 0:
                parts.append(np.ones(N * N))
                continue
            lev = wav.coefficient_level(N, self.levels)
            parts.append(vals[lev - 1].ravel())
        return np.concatenate(parts)

    def jacobi_bruteforce(self, indices=None):
        """J_lambda = alpha D_lambda + sum_{m in precond} |C~_m^-1/2 Gamma_m P_m
        W^-1 e_lambda|^2, one unit vector at a time (for ``indices`` or all)."""
        idx = np.arange(self.n) if indices is None else np.asarray(indices)
        out = np.empty(len(idx))
        for q, lam in enumerate(idx):
            l = int(np.searchsorted(self.layer_off, lam, side="right") - 1)
            N = self.N[l]
            e = np.zeros(N * N)
            e[lam - self.layer_off[l]] = 1.0
            phi = wav.idwt2(e.reshape(N, N), self.levels, self.h)
            tot = self.alpha * self.D[lam]
            for sen in self.sensors:
                if not sen["in_precond"]:
                    continue
                s, ix0, tx, jy0, ty = sen["axes"][l]
                u = geo.project_layer(phi, ix0, tx, jy0, ty)
                sl = self._measure(sen, u)
                tot += float(sl @ self._cinv(sen, sl))
            out[q] = tot
        return out

    def jacobi_separable(self):
        """Same diagonal in closed form.  A level-k coefficient (x, y) has basis
        function f_x (outer) f_y with f the 1-D k-level synthesis of a unit
        vector, and P = B_x (kron) B_y, so its Fried slopes are
        s^x_ij = dF_i sG_j, s^y_ij = sF_i dG_j with F = B_x f_x, dF_i =
        F_{i+1} - F_i, sF_i = (F_i + F_{i+1})/2 (and G likewise): the diagonal
        is a masked bilinear form in these 1-D vectors."""
        J = self.alpha * self.D.copy()
        for l, N in enumerate(self.N):
            Jl = np.zeros((N, N))
            lev = wav.coefficient_level(N, max(self.levels, 1))
            for k in range(1, max(self.levels, 1) + 1):
                M = N >> (k - 1) if self.levels else N
                Phi = np.zeros((N, M))
                for x in range(M):
                    e = np.zeros(N)
                    e[x] = 1.0
                    Phi[:, x] = wav.idwt1_multilevel(e, k, self.h) if self.levels else e
                Jk = np.zeros((M, M))
                for sen in self.sensors:
                    if not sen["in_precond"]:
                        continue
                    s, ix0, tx, jy0, ty = sen["axes"][l]
                    Bx = np.zeros((len(ix0), N))
                    Bx[np.arange(len(ix0)), ix0] += 1 - tx
                    Bx[np.arange(len(ix0)), ix0 + 1] += tx
                    By = np.zeros((len(jy0), N))
                    By[np.arange(len(jy0)), jy0] += 1 - ty
                    By[np.arange(len(jy0)), jy0 + 1] += ty
                    F = Bx @ Phi
                    G = By @ Phi
                    blk = sen["blocks"]
                    if sen["phase"]:
                        Am = np.zeros(sen["node_mask"].shape)
                        Am[sen["node_mask"]] = blk[:, 0]
                        Jk += (F ** 2).T @ Am @ (G ** 2)
                        continue
                    dF, sF = F[1:] - F[:-1], 0.5 * (F[1:] + F[:-1])
                    dG, sG = G[1:] - G[:-1], 0.5 * (G[1:] + G[:-1])
                    mask = sen["mask"]
                    if sen["cells"] is None:
                        A = np.zeros(mask.shape)
                        B = np.zeros(mask.shape)
                        C = np.zeros(mask.shape)
                        A[mask], B[mask], C[mask] = blk[:, 0], blk[:, 1], blk[:, 2]
                        Jk += (dF ** 2).T @ A @ (sG ** 2)
                        Jk += 2.0 * (dF * sF).T @ B @ (sG * dG)
                        Jk += (sF ** 2).T @ C @ (dG ** 2)
                    else:
                        for q, cm in enumerate(sen["cells"]):
                            w = cm / cm.sum()
                            sxq = dF.T @ w @ sG
                            syq = sF.T @ w @ dG
                            Jk += blk[q, 0] * sxq ** 2 + 2 * blk[q, 1] * sxq * syq \
                                + blk[q, 2] * syq ** 2
                if self.levels == 0:
                    Jl = Jk
                    continue
                sel = lev[:M, :M] == k
                Jl[:M, :M][sel] = Jk[sel]
            J[self.layer_off[l]:self.layer_off[l + 1]] += Jl.ravel()
        return J

