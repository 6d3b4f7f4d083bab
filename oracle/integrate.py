"""Linearly implicit backward-Euler integration (Section 2.1 names backward
Euler among the implicit solvers for the stiff discretised continuity
equation).  Test infrastructure only.

One step: solve (I/dt - J(n)) Delta = F(n), then n <- n + Delta.
"""

from dataclasses import dataclass

import numpy as np

from . import grid as grid_mod
from . import photolysis
from . import rates as rates_mod
from .rhs import rhs
from .jacobian import step_matrix
from .linalg import btd, btd_factor, btd_solve, dense_solve


class Problem:
    """Network + column with the grid and rate coefficients precomputed (the
    coefficients depend on T, n_gas and tau only, which are fixed)."""

    def __init__(self, net, col, spectrum=None):
        self.net = net
        self.col = col
        self.grid = grid_mod.make_grid(col, net.mass_amu)
        self.kf, self.kr = rates_mod.rates(net, self.grid)
        # spectral photolysis (Section 2.3.3): dict with absorbers, sig_ext,
        # J0, dlam, sig_ph (rows in the order of the photolysis reactions),
        # t_f, mu; None keeps the gray law
        self.spectrum = spectrum

    def lag_photolysis(self, n):
        """The photolysis coefficients of state n (spectral rates), held for
        the step that starts from n."""
        sp = self.spectrum
        photo = np.nonzero(np.asarray(self.net.rtype) == rates_mod.RT_PHOTO)[0]
        self.kf = self.kf.copy()
        self.kf[:, photo] = photolysis.spectral_rates(n, self.grid.dz, sp["absorbers"],
                                                      sp["sig_ext"], sp["J0"], sp["dlam"],
                                                      sp["sig_ph"], sp["t_f"], sp["mu"])

    def rhs(self, n):
        return rhs(self.net, self.grid, self.kf, self.kr, n)

    def step_matrix(self, n, dt):
        return step_matrix(self.net, self.grid, self.kf, self.kr, n, dt)


def be_step(prob, n, dt, solver="btd", newton_iters=1):
    """One linearly implicit BE step; newton_iters > 1 adds frozen-Jacobian
    corrections of the nonlinear BE equation n1 - n - dt F(n1) = 0.
    Returns (n_new, delta)."""
    if getattr(prob, "spectrum", None) is not None:
        prob.lag_photolysis(n)
    B, a, c = prob.step_matrix(n, dt)
    solve = btd if solver == "btd" else dense_solve
    delta = solve(B, a, c, prob.rhs(n))
    for _ in range(newton_iters - 1):
        n1 = n + delta
        resid = prob.rhs(n1) - delta / dt
        delta = delta + solve(B, a, c, resid)
    return n + delta, delta


def frozen_step(prob, n, frozen):
    """One backward-Euler step with a step matrix frozen at an earlier state
    (the factor-reusing family of stiff integrators the paper's solver
    belongs to): solve M_f Delta = F(n) with frozen = (B, a, c) of
    prob.step_matrix(n_f, dt), rates and F at n.  Returns (n_new, delta)."""
    if getattr(prob, "spectrum", None) is not None:
        prob.lag_photolysis(n)
    B, a, c = frozen
    delta = btd(B, a, c, prob.rhs(n))
    return n + delta, delta


ROS2_GAMMA = 1.0 + 1.0 / np.sqrt(2.0)


def ros2_step(prob, n, dt, stages=False):
    """One step of the two-stage, second-order, L-stable Rosenbrock method
    ROS2 (Verwer, Spee, Blom and Hundsdorfer, SIAM J. Sci. Comput. 20, 1999),
    one of the stiff integrators Section 2.1 lists for this problem, built on
    the same step matrix and block-tridiagonal solve as the backward-Euler
    step.  With gamma = 1 + 1/sqrt(2) and W = I - gamma dt J(n):
        W k1 = F(n),  W k2 = F(n + dt k1) - 2 k1,
        n_new = n + dt (3/2 k1 + 1/2 k2).
    W = gamma dt M with M = prob.step_matrix(n, gamma dt), so each stage is a
    solve with M and a division by gamma dt.  Rates (the lagged photolysis
    too) are those of n for both stages.  Returns (n_new, delta), and with
    stages=True also the two terms of delta, (3/2 dt k1, 1/2 dt k2)."""
    if getattr(prob, "spectrum", None) is not None:
        prob.lag_photolysis(n)
    gdt = ROS2_GAMMA * dt
    B, a, c = prob.step_matrix(n, gdt)
    k1 = btd(B, a, c, prob.rhs(n)) / gdt
    k2 = btd(B, a, c, prob.rhs(n + dt * k1) - 2.0 * k1) / gdt
    delta = dt * (1.5 * k1 + 0.5 * k2)
    if stages:
        return n + delta, delta, (1.5 * dt * k1, 0.5 * dt * k2)
    return n + delta, delta


def bdf2_step(prob, n, n_prev, dt, dt_prev=None):
    """One linearly implicit step of the second-order backward
    differentiation formula (BDF2, the lowest member above backward Euler of
    the BDF family that DLSODES, named in Section 2.1, integrates with).
    With the step ratio w = dt / dt_prev (dt_prev: the step that led from
    n_prev to n; None = dt) the variable-step formula is
        n_new - (1+w)^2/(1+2w) n + w^2/(1+2w) n_prev = (1+w)/(1+2w) dt F(n_new),
    with F(n_new) linearised about n (one Newton iteration from n).  With
    h = (1+w)/(1+2w) dt and Delta = n_new - n this is the backward-Euler
    system of step h with a history term on the right-hand side:
        (I/h - J(n)) Delta = F(n) + w^2/(1+2w) (n - n_prev) / h.
    At w = 1: h = 2 dt/3 and the history term (n - n_prev)/(2 dt).
    Returns (n_new, delta)."""
    if getattr(prob, "spectrum", None) is not None:
        prob.lag_photolysis(n)
    w = 1.0 if dt_prev is None else dt / dt_prev
    h = (1.0 + w) / (1.0 + 2.0 * w) * dt
    B, a, c = prob.step_matrix(n, h)
    hist = w * w / (1.0 + 2.0 * w) * (n - n_prev) / h
    delta = btd(B, a, c, prob.rhs(n) + hist)
    return n + delta, delta


def fixed_schedule(nsteps=200, dt0=1.0e-8, growth=1.2):
    """dt_j = dt0 * growth^j, j = 0 .. nsteps-1."""
    return [dt0 * growth ** j for j in range(nsteps)]


def run_fixed(prob, n0, schedule, solver="btd"):
    n = n0.copy()
    for dt in schedule:
        n, _ = be_step(prob, n, dt, solver)
    return n


@dataclass
class SteadyResult:
    n: np.ndarray
    t: float
    dt: float
    steps: int
    rejects: int
    converged: bool
    clipped: float
    history: list


def steady_state(prob, n0, tol_rel=1.0e-4, y_floor=1.0e-30, y_sig=1.0e-10,
                 t_end=1.0e12, dt0=1.0e-8, max_steps=5000,
                 max_consec_rejects=30, use_mix_rule=True, method="be", y_neg=1.0e-6):
    """Adaptive driver to steady state; each step is a backward-Euler step
    (method "be") or a ROS2 step (method "ros2"), with the same control.

    * Reject a step (dt <- dt/2) if it is not finite or if a species whose
      mixing ratio exceeded y_sig turns more negative than -y_neg in mixing
      ratio (y_neg = 0: any negative); after more than max_consec_rejects
      consecutive rejections give up (not converged).  A smaller overshoot
      is clipped like any other negative: it adds at most y_neg of the
      layer's gas density to that species in that step.
    * On acceptance clip negative densities to zero (the clipped amount is
      recorded) and adapt dt from the largest relative change of the
      species above y_sig, c = max |n1 - n0| / max(n0, n1):
      dt <- 2 dt if c < 0.5, 1.2 dt if c < 0.9, else 0.7 dt.
    * Converged when the largest relative change max |Delta n| / n over
      mixing ratios above y_floor is below tol_rel while dt is at least the
      longest layer mixing time dzh^2/(K + D) (Section 3.2: the variation
      timescale must exceed the layer mixing timescale; Section 2 checks
      convergence as a relative change between iterations), or when
      t >= t_end.
    """
    ngas = prob.grid.ngas[:, None]
    mix = prob.grid.mix_time if use_mix_rule else 0.0
    n = n0.copy()
    t, dt = 0.0, dt0
    steps = rejects = consec = 0
    clipped = 0.0
    hist = []
    converged = False
    step = {"be": be_step, "ros2": ros2_step}[method]
    while steps < max_steps:
        n_new, delta = step(prob, n, dt)
        sig = n > y_sig * ngas
        if not np.all(np.isfinite(n_new)) or np.any(sig & (n_new < -y_neg * ngas)):
            rejects += 1
            consec += 1
            dt *= 0.5
            if consec > max_consec_rejects:
                break
            continue
        consec = 0
        neg = n_new < 0.0
        clipped += float(-n_new[neg].sum())
        n_new[neg] = 0.0
        keep = n_new > y_floor * ngas
        rel = float(np.max(np.abs(n_new[keep] - n[keep]) / n_new[keep])) if keep.any() else 0.0
        ctl = n_new > y_sig * ngas
        big = np.maximum(n_new[ctl], n[ctl])
        c = float(np.max(np.abs(n_new[ctl] - n[ctl]) / big)) if ctl.any() else 0.0
        t += dt
        steps += 1
        n = n_new
        hist.append((t, dt, rel, c))
        if (rel < tol_rel and dt >= mix) or t >= t_end:
            converged = True
            break
        dt *= 2.0 if c < 0.5 else (1.2 if c < 0.9 else 0.7)
    return SteadyResult(n=n, t=t, dt=dt, steps=steps, rejects=rejects,
                        converged=converged, clipped=clipped, history=hist)


def newton_held(prob, n, dt, held, newton_tol=1.0e-3, max_newton=4, y_sig=1.0e-10):
    """Modified Newton on the backward-Euler equation n1 - n - dt F(n1) = 0
    with a step matrix factored earlier (held = (factors, a, c) of
    step_matrix(n_f, dt_f)): from Delta = 0,
        Delta += M_f^-1 (F(n + Delta) - Delta / dt),
    until a correction is at most newton_tol of every new density whose
    mixing ratio exceeds y_sig (converged), or a correction is not below half
    the previous one, or max_newton corrections are spent, or the iterate is
    not finite (failed).  Returns (Delta, converged, corrections)."""
    ngas = prob.grid.ngas[:, None]
    fac, a, c = held
    delta = np.zeros_like(n)
    prev = np.inf
    for it in range(1, max_newton + 1):
        resid = prob.rhs(n + delta) - delta / dt
        corr = btd_solve(fac, a, c, resid)
        delta = delta + corr
        n1 = n + delta
        if not np.all(np.isfinite(n1)):
            return delta, False, it
        sig = np.abs(n1) > y_sig * ngas
        size = float(np.max(np.abs(corr[sig]) / np.abs(n1[sig]))) if sig.any() else 0.0
        if size <= newton_tol:
            return delta, True, it
        if size > 0.5 * prev:
            return delta, False, it
        prev = size
    return delta, False, max_newton


def fixed_dt_reuse(prob, n0, dt, nsteps, newton_tol=1.0e-3, max_newton=4, max_age=20,
                   y_sig=1.0e-10):
    """nsteps backward-Euler steps of one size dt that keep the step matrix
    across steps (the chord / modified-Newton corrector of the DLSODES
    family): a step on a fresh factorisation of M = I/dt - J(n) takes the
    first Newton iterate (the linearly implicit step); a step on the held
    factorisation (of an earlier state) iterates newton_held to convergence;
    when that fails, or the factorisation has served max_age steps, the step
    is taken again on a fresh one.  No clipping, no rejection.  Returns
    (n, factorizations, newton corrections)."""
    n = n0.copy()
    held = None
    age = nfact = ncorr = 0
    for _ in range(nsteps):
        if held is not None and age < max_age:
            delta, ok, it = newton_held(prob, n, dt, held, newton_tol, max_newton, y_sig)
            ncorr += it
            if ok:
                n = n + delta
                age += 1
                continue
        B, a, c = prob.step_matrix(n, dt)
        held = (btd_factor(B, a, c), a, c)
        nfact += 1
        age = 1
        n = n + btd_solve(held[0], a, c, prob.rhs(n))
    return n, nfact, ncorr


@dataclass
class ReuseResult(SteadyResult):
    factorizations: int = 0
    newton_iters: int = 0


def steady_state_reuse(prob, n0, tol_rel=1.0e-4, y_floor=1.0e-30, y_sig=1.0e-10,
                       t_end=1.0e12, dt0=1.0e-8, max_steps=5000, max_consec_rejects=30,
                       use_mix_rule=True, newton_tol=1.0e-3, max_newton=4, max_age=20,
                       reuse_ratio=1.3, y_neg=1.0e-6):
    """The adaptive steady-state driver with the step matrix kept across
    steps, after the corrector of the DLSODES family Section 2.1 names
    (modified Newton on the backward-Euler equation, one factorisation
    serving several steps).

    * A step of size dt at state n solves n1 - n - dt F(n1) = 0.  With a
      freshly factored matrix M = I/dt - J(n) it takes the first Newton
      iterate, Delta = M^-1 F(n): the linearly implicit step of the plain
      driver.  With a held matrix (factored at an earlier state and step
      size dt_f) it iterates Delta += M_f^-1 (F(n + Delta) - Delta/dt) from
      Delta = 0 (newton_held: converged once a correction is at most
      newton_tol of every new density with mixing ratio above y_sig; a
      correction not below half the previous one, a non-finite iterate or
      max_newton corrections end the attempt), and a failed attempt is
      retried with a fresh matrix (not a rejection).
    * The held matrix serves while dt / dt_f lies in [1/reuse_ratio,
      reuse_ratio] and it has served fewer than max_age steps; otherwise a
      new one is factored at the current state and dt.
    * Acceptance, clipping, the dt rule and the convergence test are those
      of steady_state (a rejection halves dt, so it refactors).
    """
    ngas = prob.grid.ngas[:, None]
    mix = prob.grid.mix_time if use_mix_rule else 0.0
    n = n0.copy()
    t, dt = 0.0, dt0
    steps = rejects = consec = nfact = nnewton = 0
    clipped = 0.0
    hist = []
    converged = False
    held = None            # (factors, a, c, dt_f, age)
    while steps < max_steps:
        fresh = held is None or not (1.0 / reuse_ratio <= dt / held[3] <= reuse_ratio) \
            or held[4] >= max_age
        if fresh:
            B, a, c = prob.step_matrix(n, dt)
            held = [btd_factor(B, a, c), a, c, dt, 0]
            nfact += 1
            delta = btd_solve(held[0], a, c, prob.rhs(n))
            ok = bool(np.all(np.isfinite(delta)))
        else:
            delta, ok, it = newton_held(prob, n, dt, held[:3], newton_tol, max_newton, y_sig)
            nnewton += it
            if not ok:
                held = None        # retry this step with a fresh matrix
                continue
        n_new = n + delta
        sig = n > y_sig * ngas
        if not ok or not np.all(np.isfinite(n_new)) or np.any(sig & (n_new < -y_neg * ngas)):
            rejects += 1
            consec += 1
            dt *= 0.5
            if consec > max_consec_rejects:
                break
            continue
        consec = 0
        held[4] += 1
        neg = n_new < 0.0
        clipped += float(-n_new[neg].sum())
        n_new[neg] = 0.0
        keep = n_new > y_floor * ngas
        rel = float(np.max(np.abs(n_new[keep] - n[keep]) / n_new[keep])) if keep.any() else 0.0
        ctl = n_new > y_sig * ngas
        big = np.maximum(n_new[ctl], n[ctl])
        c = float(np.max(np.abs(n_new[ctl] - n[ctl]) / big)) if ctl.any() else 0.0
        t += dt
        steps += 1
        n = n_new
        hist.append((t, dt, rel, c))
        if (rel < tol_rel and dt >= mix) or t >= t_end:
            converged = True
            break
        dt *= 2.0 if c < 0.5 else (1.2 if c < 0.9 else 0.7)
    return ReuseResult(n=n, t=t, dt=dt, steps=steps, rejects=rejects, converged=converged,
                       clipped=clipped, history=hist, factorizations=nfact,
                       newton_iters=nnewton)
