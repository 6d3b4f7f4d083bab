"""The Lagrangian parcel scheme of the paper's own model (Section 2, the
parcel figure; Section 2.1, molecular diffusion as a pseudo-reaction).
Test infrastructure only.

One global iteration tracks an air parcel from the bottom of the column to
the top and back down.  At each layer it visits the parcel takes the layer's
temperature and gas density (its mixing ratios carried over), stays for the
layer's residence time, and its composition evolves by the layer's chemistry
plus molecular diffusion with the neighbouring layers of the current
profile; the composition it leaves with becomes the profile at that layer.
Eddy mixing is the parcel's motion itself, so the eddy terms of the
transport do not appear (Section 2.1).  The profiles of successive global
iterations are compared for convergence (Section 2).

Readings (the paper gives none of these numbers):
* residence time at layer k: the layer's eddy mixing time dz_k^2 / K_k;
* the stiff integration of a visit: linearly implicit backward-Euler steps
  (one of the solvers Section 2.1 lists; the paper's own is the adaptive
  DLSODES) under the step control of the column's steady-state driver,
  each solving the dense S x S system of the layer
  (I/dt - J_chem - D_self) Delta = F; a visit starts with the step size the
  previous one ended on;
* molecular diffusion at layer k: the molecular-diffusion part of the
  discretised transport (Eq. discrete_continuity with Eq. dzz) as a
  pseudo-reaction: its self-coefficient removes the diffusing molecule from
  the parcel where it is a loss (negative), and every gain, the exchange
  with the profile's densities at k-1 and k+1 and a positive
  self-coefficient (the drift of species heavier than the mean can give
  one) applied to the profile's own density at k, re-enters as a fixed
  source during the visit; at a profile that the parcel reproduces these
  are the column's transport terms;
* the path visits layers 0, 1, ..., N-1, N-2, ..., 0 (the top once);
* convergence: the largest relative change of the mixing ratios above
  y_floor between the profiles of successive global iterations is below
  tol (0.1 % in the paper).
"""

from dataclasses import dataclass, replace

import numpy as np

from .jacobian import chem_jacobian, transport_coefficients
from .rhs import chem_rhs, reaction_rates


def diffusion_coefficients(grid):
    """(lower, diag, upper) [N, S] of the molecular-diffusion part of the
    transport alone: the column's transport coefficients with K = 0."""
    g = replace(grid, Kh=np.zeros_like(grid.Kh), v_top=None, v_dep=None, phi_surf=None)
    return transport_coefficients(g)


def residence_times(col, grid):
    """dz_k^2 / K_k, the eddy mixing time of each layer (reading)."""
    K = np.asarray(col.Kzz, float)
    return grid.dz ** 2 / K


def path(N):
    """Layer sequence of one global iteration: bottom to top and back."""
    return list(range(N)) + list(range(N - 2, -1, -1))


def layer_rhs(prob, k, p, prof, diff):
    """F of the parcel p [S] at layer k: chemistry with the layer's rate
    coefficients, the diffusion loss on the parcel, and the diffusion gains
    from the profile."""
    lower, diag, upper = diff
    w = reaction_rates(prob.net, prob.kf[k:k + 1], prob.kr[k:k + 1], p[None, :])
    loss = np.minimum(diag[k], 0.0)
    f = chem_rhs(prob.net, w, p.shape[0])[0] + loss * p + (diag[k] - loss) * prof[k]
    if k >= 1:
        f = f + lower[k] * prof[k - 1]
    if k + 1 < prof.shape[0]:
        f = f + upper[k] * prof[k + 1]
    return f


def layer_matrix(prob, k, p, dt, diff):
    """M = I/dt - dF/dp at layer k (dense S x S): the chemistry and the
    diffusion loss depend on the parcel."""
    J = chem_jacobian(prob.net, prob.kf[k:k + 1], prob.kr[k:k + 1], p[None, :])[0]
    S = p.shape[0]
    return np.eye(S) / dt - J - np.diag(np.minimum(diff[1][k], 0.0))


def visit(prob, k, p, prof, diff, t_res, dt0, y_sig=1.0e-10, max_consec_rejects=30):
    """The parcel's composition after t_res at layer k, integrated by
    linearly implicit backward-Euler steps with the step control of the
    column's steady-state driver (integrate.steady_state) with no overshoot
    tolerance (y_neg = 0) inside the window:
    a step that is not finite or turns a species above mixing ratio y_sig
    negative is taken again at half the size; an accepted step clips
    negatives to zero and sets the next size by the control change c
    (x2 if c < 0.5, x1.2 if c < 0.9, else x0.7); the last step ends at
    t_res.  dt0 is the first step's size.  Returns (p, the size the next
    step would take, steps, rejections, clipped density)."""
    ngas = prob.grid.ngas[k]
    t, dt = 0.0, dt0
    steps = rejects = consec = 0
    clipped = 0.0
    while t < t_res:
        h = min(dt, t_res - t)
        delta = np.linalg.solve(layer_matrix(prob, k, p, h, diff),
                                layer_rhs(prob, k, p, prof, diff))
        q = p + delta
        if not np.all(np.isfinite(q)) or np.any((p > y_sig * ngas) & (q < 0.0)):
            rejects += 1
            consec += 1
            if consec > max_consec_rejects:
                raise RuntimeError(f"parcel visit at layer {k}: step size collapsed")
            dt = 0.5 * h
            continue
        consec = 0
        neg = q < 0.0
        clipped += float(-q[neg].sum())
        q[neg] = 0.0
        ctl = q > y_sig * ngas
        big = np.maximum(q[ctl], p[ctl])
        c = float(np.max(np.abs(q[ctl] - p[ctl]) / big)) if ctl.any() else 0.0
        t += h
        steps += 1
        p = q
        dt = h * (2.0 if c < 0.5 else (1.2 if c < 0.9 else 0.7))
    return p, dt, steps, rejects, clipped


@dataclass
class ParcelResult:
    n: np.ndarray
    iterations: int
    converged: bool
    history: list
    steps: int = 0
    rejects: int = 0
    clipped: float = 0.0


def global_iteration(prob, prof, diff, t_res, dt0=1.0e-8):
    """One bottom-to-top-to-bottom pass; returns (new profile, steps,
    rejections, clipped density).  The first visit starts with step dt0,
    each later one with the step size the previous visit ended on, at most
    its own residence time."""
    ngas = prob.grid.ngas
    prof = prof.copy()
    seq = path(prob.grid.N)
    p = prof[seq[0]].copy()
    dt = dt0
    steps = rejects = 0
    clipped = 0.0
    for i, k in enumerate(seq):
        if i > 0:
            p = p * (ngas[k] / ngas[seq[i - 1]])   # same mixing ratios, new layer
        p, dt, st, rj, cl = visit(prob, k, p, prof, diff, t_res[k], min(dt, t_res[k]))
        steps += st
        rejects += rj
        clipped += cl
        prof[k] = p
    return prof, steps, rejects, clipped


def run(prob, n0, max_iter=50, tol=1e-3, y_floor=1e-30, dt0=1.0e-8):
    """Global iterations from profile n0 until the mixing ratios change by
    less than tol between successive iterations (or max_iter)."""
    diff = diffusion_coefficients(prob.grid)
    t_res = residence_times(prob.col, prob.grid)
    ngas = prob.grid.ngas[:, None]
    prof = n0.copy()
    hist = []
    steps = rejects = 0
    clipped = 0.0
    for it in range(1, max_iter + 1):
        new, st, rj, cl = global_iteration(prob, prof, diff, t_res, dt0)
        steps += st
        rejects += rj
        clipped += cl
        keep = new > y_floor * ngas
        change = float(np.max(np.abs(new[keep] - prof[keep]) / new[keep])) if keep.any() else 0.0
        hist.append(change)
        prof = new
        if change < tol:
            return ParcelResult(prof, it, True, hist, steps, rejects, clipped)
    return ParcelResult(prof, max_iter, False, hist, steps, rejects, clipped)
