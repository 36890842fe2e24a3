"""Element-wise comparison of GPU records with oracle records.

Relative errors: value |dV| / |V_ref|; gradient |dG| / max(|G_ref|, eta S_G);
Hessian |dH|_F / max(|H_ref|_F, eta S_H), where S_G, S_H are the sums of
per-triangle term norms reported by the oracle (the scale of the
cancellation inside the sum) and eta = 1e-4.
"""
import numpy as np

TOL_V, TOL_G, TOL_H, ETA = 1e-4, 1e-3, 5e-3, 1e-4


def hess_fro(h6):
    h6 = np.asarray(h6)
    return np.sqrt(h6[..., 0] ** 2 + h6[..., 3] ** 2 + h6[..., 5] ** 2 +
                   2 * (h6[..., 1] ** 2 + h6[..., 2] ** 2 + h6[..., 4] ** 2))


def rel_errors(value, grad, hess, ref):
    """Per record and channel: (err_V, err_G, err_H, floor_bound_G, floor_bound_H)."""
    V, G, H, st = ref["value"], ref["grad"], ref["hess"], ref["stats"]
    SG = np.stack([st[:, 3], st[:, 5]], 1)
    SH = np.stack([st[:, 4], st[:, 6]], 1)
    dv = np.abs(value - V)
    vden = np.abs(V)
    ev = np.where(vden > 0, dv / np.where(vden > 0, vden, 1), np.where(dv == 0, 0.0, np.inf))
    ng = np.linalg.norm(G, axis=-1)
    dg = np.linalg.norm(grad - G, axis=-1)
    gden = np.maximum(ng, ETA * SG)
    eg = np.where(gden > 0, dg / np.where(gden > 0, gden, 1), np.where(dg == 0, 0.0, np.inf))
    nh = hess_fro(H)
    dh = hess_fro(hess - H)
    hden = np.maximum(nh, ETA * SH)
    eh = np.where(hden > 0, dh / np.where(hden > 0, hden, 1), np.where(dh == 0, 0.0, np.inf))
    return ev, eg, eh, ng < ETA * SG, nh < ETA * SH


def assert_parity(value, grad, hess, ref, label=""):
    ev, eg, eh, fg, fh = rel_errors(value, grad, hess, ref)
    msg = (f"{label}: max rel err value {ev.max():.2e} (tol {TOL_V}), grad {eg.max():.2e} (tol {TOL_G}), "
           f"hess {eh.max():.2e} (tol {TOL_H}); floor binds on {fg.mean():.1%} grad / {fh.mean():.1%} hess")
    print(msg, flush=True)
    assert ev.max() <= TOL_V and eg.max() <= TOL_G and eh.max() <= TOL_H, msg
    return ev, eg, eh
