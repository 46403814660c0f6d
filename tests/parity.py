"""Error measures and parity bars of the HIP path against the FP64 oracle.

Every bar is computed from the oracle's values and the stated tolerances
alone, never from the GPU's output.

* states: per window unit, ||x_gpu - x_ref||_inf / max(||x_ref||_inf, 1e-6)
  <= 1e-4 over the unit's h states.
* gradients: per particle, the normwise error ||g_gpu - g_ref||_2 /
  ||g_ref||_2 <= 1e-3 wherever the gradient is not dominated by
  cancellation, i.e. wherever the per-window terms it sums (w_k dl_kj/dtheta
  for g_obs, seed_kj dg_kj/dtheta for g_con) have norms adding up to at most
  2 ||g_ref||.  Where they add up to more (near an optimum; the single
  pendulum's dl/dm is exactly 0), the bar is 1e-3 sum_kj ||term_kj||, the
  error that FP32 rounding of each term implies.
  A constraint term is proportional to its defect e = (S - s_end) u twice
  (through dg_def/ds_end and through the seed lam + c g_def), so an error
  in the end state that the state tolerance allows moves it by up to three
  times that error relative to e.  The g_con bar therefore adds
  3 sum_kj ||term_kj|| dhat_kj with dhat_kj = min(1, 1e-4 max|s_end_ref|
  sqrt(d_s) / ||e_ref||): the defect's relative error the state tolerance
  permits, from the oracle's end states.
* S_dot: per particle ||dS_gpu - dS_ref|| / ||dS_ref|| <= 1e-3.
* window log-likelihoods: the error the state tolerance implies,
  sum_t,d |r| w 1e-4 max(||x||_inf, 1e-6), plus 1e-9 |l| for the FP64
  sums (r = residual, w = 1/sigma_obs).
* bandwidth: exact median (the same FP64 arithmetic on both sides).
* phi: FP32 sums of N terms, |d phi| <= 1e-4 (1/N) sum_j k_ij (|G_j| +
  |grad k|) per component.
"""
from __future__ import annotations

import numpy as np

STATE_TOL = 1e-4
GRAD_TOL = 1e-3
CANCEL_RATIO = 2.0


def state_rel_err(pb, traj_gpu, traj_ref):
    """Per window unit relative error of the visited states [N, K, n_s]."""
    N, K = traj_ref.shape[:2]
    tg = traj_gpu.reshape(N, K, pb.n_s, pb.h, pb.d_s)
    tr = traj_ref.reshape(N, K, pb.n_s, pb.h, pb.d_s)
    err = np.abs(tg - tr).max(axis=(3, 4))
    scale = np.maximum(np.abs(tr).max(axis=(3, 4)), 1e-6)
    return err / scale


def observed_err_ratio(pb, tobs_gpu, x_ref, traj_ref):
    """Per window unit error of the observed quantities [N, K, n_s] as a
    fraction of what the state tolerance permits.  Components of the state
    (planar models, the hinge angle) move by at most the state error; a
    box-frame point p moves by sum_j |dq_j| |p - o_j|, with |p - o_j| at most
    the reach R of the chain (every DH offset, the flange offset and the
    1 m to the farthest observed point), so its bar is n_dof R times the
    state bar."""
    N, K = traj_ref.shape[:2]
    tr = traj_ref.reshape(N, K, pb.n_s, pb.h, pb.d_s)
    scale = np.maximum(np.abs(tr).max(axis=(3, 4)), 1e-6)
    gain = 1.0
    if pb.kind in (5, 6):
        a = pb.arm
        reach = np.abs(a["dh_a"]).sum() + np.abs(a["dh_d"]).sum() + abs(a["flange_d"]) + 1.0
        gain = pb.n_dof * reach
    err = np.abs(tobs_gpu - x_ref).reshape(N, K, pb.n_s, pb.h, pb.d_x).max(axis=(3, 4))
    return err / (STATE_TOL * scale * gain)


def end_state_rel_err(es_gpu, es_ref):
    """Per window unit relative error of the window end states."""
    return np.abs(es_gpu - es_ref).max(axis=3) / np.maximum(np.abs(es_ref).max(axis=3), 1e-6)


def ll_tolerance(pb, obs, traj_ref, ll_ref):
    N, K = traj_ref.shape[:2]
    x = traj_ref[..., pb.obs_index]  # [N, K, T, d_x]
    r = (obs[None] - x) * pb.w_x
    tr = traj_ref.reshape(N, K, pb.n_s, pb.h, pb.d_s)
    scale = np.maximum(np.abs(tr).max(axis=(3, 4)), 1e-6)
    per = (np.abs(r) * pb.w_x).reshape(N, K, pb.n_s, pb.h, pb.d_x).sum(axis=(3, 4))
    return STATE_TOL * per * scale + 1e-9 * np.abs(ll_ref)


def normwise(a, b):
    a = a.reshape(a.shape[0], -1)
    b = b.reshape(b.shape[0], -1)
    den = np.maximum(np.linalg.norm(b, axis=1), 1e-30)
    return np.linalg.norm(a - b, axis=1) / den


def defect_bound(pb, ref, S):
    """dhat_kj: the relative error of each defect vector e = (S - s_end) u
    that end states within the state tolerance permit, from the oracle's
    end states [n, K, n_s - 1]."""
    es = ref["end_states"][:, :, : pb.n_s - 1]
    e = (S - es) * pb.u
    allowed = STATE_TOL * np.maximum(np.abs(es).max(axis=3), 1e-6) * np.sqrt(pb.d_s) * np.abs(pb.u).max()
    return np.minimum(1.0, allowed / np.maximum(np.linalg.norm(e, axis=3), 1e-30))


def grad_bar(ref, kind, pb=None, S=None):
    """Per-particle bar of a theta gradient channel ("obs" or "con") and
    the facts it rests on: (bar, ||g_ref||, sum_kj ||term_kj||, cancel)."""
    if kind == "obs":
        terms = ref["wk"][:, :, None, None] * ref["dl_dtheta_unit"]
        g_ref = ref["g_obs"]
    else:
        terms = ref["dcon_dtheta_unit"]
        g_ref = ref["g_con"]
    tn = np.linalg.norm(terms, axis=3)
    tsum = tn.sum(axis=(1, 2))
    nrm = np.linalg.norm(g_ref, axis=1)
    cancel = tsum > CANCEL_RATIO * nrm
    bar = GRAD_TOL * np.where(cancel, tsum, nrm)
    if kind == "con" and pb is not None and pb.n_s > 1:
        dh = defect_bound(pb, ref, S)
        bar = bar + 3.0 * (tn[:, :, : pb.n_s - 1] * dh).sum(axis=(1, 2))
    return bar, nrm, tsum, cancel


def grad_check(g_gpu, ref, kind, pb=None, S=None):
    """Per-particle comparison of a theta gradient with the oracle's.

    Returns a dict: `ratio` (error / bar, <= 1 passes), `normwise`
    (||dg|| / ||g_ref||), `terms` (sum_kj ||term_kj|| / ||g_ref||) and
    `cancel` (the term-sum bar applies)."""
    g_ref = ref["g_obs"] if kind == "obs" else ref["g_con"]
    bar, nrm, tsum, cancel = grad_bar(ref, kind, pb, S)
    err = np.linalg.norm(g_gpu - g_ref, axis=1)
    return dict(ratio=err / np.maximum(bar, 1e-300), normwise=err / np.maximum(nrm, 1e-300),
                terms=tsum / np.maximum(nrm, 1e-300), cancel=cancel)


def update_check(new_gpu, old, new_ref, grad_ref=None, lr=None):
    """Per-particle error of an update stored in FP32, returned as error /
    bar.  The bar is 1e-3 of the oracle's increment, or, for a plain
    gradient step x += lr * g with per-component step sizes, the gradient's
    own bar carried through the step, 1e-3 max|lr| ||g_ref|| (which bounds
    ||lr (g - g_ref)|| whenever g meets its bar); plus the rounding of
    storing the updated values in FP32 (2^-24 relative per element, bounded
    normwise by 2^-23 ||new_ref||)."""
    n = new_ref.shape[0]
    d_g = (new_gpu - old).reshape(n, -1)
    d_r = (new_ref - old).reshape(n, -1)
    if grad_ref is None:
        inc = GRAD_TOL * np.linalg.norm(d_r, axis=1)
    else:
        inc = GRAD_TOL * np.max(np.abs(lr)) * np.linalg.norm(grad_ref.reshape(n, -1), axis=1)
    bar = inc + 2.0 ** -23 * np.linalg.norm(new_ref.reshape(n, -1), axis=1)
    return np.linalg.norm(d_g - d_r, axis=1) / np.maximum(bar, 1e-300)


def phi_scale(theta, G, rho, h, sel=None):
    """(1/N) sum_j k_ij (|G_j| + |grad k|) per component, the phi bar's scale."""
    ti = theta if sel is None else theta[sel]
    d = (ti[:, None, :] - theta[None, :, :]) / rho
    k = np.exp(-(d ** 2).sum(-1) / h)
    gk = k[:, :, None] * 2.0 / h * np.abs(d) / rho
    return (k[:, :, None] * np.abs(G)[None, :, :] + gk).mean(axis=1)
