"""ORACLE (test infrastructure only): (preconditioned) conjugate gradients for
the normal equations, plain FP64.

The paper solves eq. (19) with CG or with PCG and the modified Jacobi
preconditioner, a fixed number of iterations, and a warm restart from the
previous time step's reconstruction (Sec. 5.1).  This is the standard
Hestenes-Stiefel recurrence with no tolerance stop: it halts early only on
breakdown (rho = 0 exactly: converged; p^T A p <= 0 or non-finite: broken).
"""
import numpy as np

STATUS_OK, STATUS_CONVERGED, STATUS_BREAKDOWN = 0, 1, -1


def pcg(apply_A, b, n_iter, x0=None, jacobi=None, true_residuals=False):
    """Returns (x, info).  ``jacobi`` is the preconditioner diagonal (None for
    plain CG).  info: rho history, step sizes, status and, if asked, the true
    residual norms |b - A x_i| for i = 0..n_iter; "rnorm" holds the recursive
    residual norms |r_i|."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    r = b - apply_A(x) if x0 is not None else b.copy()
    z = r / jacobi if jacobi is not None else r.copy()
    p = z.copy()
    rho = float(r @ z)
    info = {"rho": [rho], "alpha": [], "beta": [], "status": STATUS_OK, "iters": 0,
            "rnorm": [float(np.linalg.norm(r))]}
    if true_residuals:
        info["resid"] = [float(np.linalg.norm(b - apply_A(x)))]
    for i in range(n_iter):
        if rho == 0.0:
            info["status"] = STATUS_CONVERGED
            break
        q = apply_A(p)
        pq = float(p @ q)
        if not np.isfinite(pq) or pq <= 0.0:
            info["status"] = STATUS_BREAKDOWN
            break
        a = rho / pq
        x = x + a * p
        r = r - a * q
        z = r / jacobi if jacobi is not None else r.copy()
        rho_new = float(r @ z)
        beta = rho_new / rho
        p = z + beta * p
        rho = rho_new
        info["alpha"].append(a)
        info["beta"].append(beta)
        info["rho"].append(rho)
        info["rnorm"].append(float(np.linalg.norm(r)))
        info["iters"] = i + 1
        if true_residuals:
            info["resid"].append(float(np.linalg.norm(b - apply_A(x))))
    return x, info
