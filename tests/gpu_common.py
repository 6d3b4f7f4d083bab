"""Shared helpers for the GPU parity tests: build the same problem on both
sides (oracle on the CPU, HIP library on the GPU) from the same seeded
inputs."""

import numpy as np
import torch

import synth
from oracle import integrate

EPS = np.finfo(float).eps


def dev():
    return torch.device("cuda:0")


def make_pair(net, col, precision=0):
    import paper_2512_06729_amd as xod
    stream = torch.cuda.current_stream().cuda_stream
    gnet = xod.Network(net)
    gcol = xod.Column(gnet, col, precision=precision, stream=stream)
    prob = integrate.Problem(net, col)
    return prob, gnet, gcol


def config_pair(c, precision=0):
    net, col = synth.make_config(c)
    return (net, col) + make_pair(net, col, precision)


def gpu_rates(gcol):
    import paper_2512_06729_amd as xod
    kf = torch.empty(gcol.N * gcol.R, dtype=torch.float64, device=dev())
    kr = torch.empty_like(kf)
    xod.xod_rates(gcol, kf, kr)
    return kf, kr


def to_np(t, shape=None):
    torch.cuda.synchronize()
    a = t.detach().cpu().numpy()
    return a.reshape(shape) if shape is not None else a


def gpu_blocks(gcol, kf, kr, n_np, dt):
    import paper_2512_06729_amd as xod
    N, S, ld = gcol.N, gcol.S, gcol.ld
    n = torch.from_numpy(np.ascontiguousarray(n_np)).to(dev()).reshape(-1)
    B = torch.empty(N * ld * ld, dtype=torch.float64, device=dev())
    a = torch.empty(N * ld, dtype=torch.float64, device=dev())
    c = torch.empty_like(a)
    xod.xod_jacobian(gcol, kf, kr, n, dt, B, a, c)
    return n, B, a, c


def gpu_solve(gcol, kf, kr, n_np, dt, rhs_np):
    """Factor the step matrix at (n, dt) on the GPU and solve for rhs."""
    import paper_2512_06729_amd as xod
    n, B, a, c = gpu_blocks(gcol, kf, kr, n_np, dt)
    piv = torch.empty(gcol.N * gcol.ld, dtype=torch.int32, device=dev())
    xod.xod_btd_factor(gcol, B, a, c, piv)
    x = torch.from_numpy(np.ascontiguousarray(rhs_np)).to(dev()).reshape(-1)
    xod.xod_btd_solve(gcol, B, a, c, piv, x)
    return to_np(x, (gcol.N, gcol.S))


def assert_solve_agrees(x, ref, rel=1e-10, frac=1e-6):
    """Per layer: |x - ref| <= rel * max(|ref|, frac * max_layer |ref|).

    Entries far below their layer's largest are only determined to about
    eps * cond(M) * max |ref| by any backward-stable solver (two LAPACK-based
    solvers in the oracle already differ there), so they are held to the
    same absolute floor as the small-but-resolved ones."""
    lm = np.abs(ref).max(axis=-1, keepdims=True)
    allowed = rel * np.maximum(np.abs(ref), frac * lm)
    worst = float(np.max(np.abs(x - ref) / (allowed + 1e-300)))
    assert worst <= 1.0, f"solve disagreement {worst:.3e} x allowed"


def assert_state_agrees(n, ref, delta, rel=1e-10, frac=1e-6):
    """A stepped state: the increment is held as in assert_solve_agrees, plus
    the rounding of n0 + delta itself (a few eps of |n|)."""
    lm = np.abs(delta).max(axis=-1, keepdims=True)
    allowed = rel * np.maximum(np.abs(delta), frac * lm) + 4 * EPS * np.abs(ref)
    ratio = np.abs(n - ref) / (allowed + 1e-300)
    k, y = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
    worst = float(ratio[k, y])
    msg = (f"state disagreement {worst:.3e} x allowed at layer {k} species {y}: "
           f"n {n[k, y]:.17e} ref {ref[k, y]:.17e} delta {delta[k, y]:.3e} "
           f"layer max |delta| {lm[k, 0]:.3e}")
    print(msg)
    assert worst <= 1.0, msg


def block_kappa(prob, n, dt):
    """Largest 1-norm condition number over the layers of the diagonal step
    blocks B_k = I/dt - dF_k/dn_k at state n (the oracle's blocks), from
    LAPACK's estimator on each block's LU factors."""
    import scipy.linalg
    B, a, c = prob.step_matrix(n, dt)
    worst = 1.0
    for k in range(B.shape[0]):
        lu, _ = scipy.linalg.lu_factor(B[k])
        rcond, info = scipy.linalg.lapack.dgecon(lu, np.abs(B[k]).sum(axis=0).max(), norm="1")
        worst = max(worst, 1.0 / rcond if rcond > 0 else np.inf)
    return float(worst)


def assert_state_agrees_kappa(n, ref, delta, kappa, rel=1e-10, c=10.0):
    """A stepped state held to the forward-error bound of a backward-stable
    solve: per layer, |n - ref| <= rel |delta| + c kappa eps max_layer |delta|
    (+ the rounding of n0 + delta).  The per-layer floor of
    assert_state_agrees is this bound at kappa ~ 1; with the stiff blocks of
    large steps the floor grows with the blocks' condition number kappa."""
    lm = np.abs(delta).max(axis=-1, keepdims=True)
    allowed = rel * np.abs(delta) + c * kappa * EPS * lm + 4 * EPS * np.abs(ref)
    ratio = np.abs(n - ref) / (allowed + 1e-300)
    k, y = np.unravel_index(int(np.argmax(ratio)), ratio.shape)
    worst = float(ratio[k, y])
    msg = (f"state disagreement {worst:.3e} x allowed (kappa {kappa:.2e}) at layer {k} "
           f"species {y}: n {n[k, y]:.17e} ref {ref[k, y]:.17e} delta {delta[k, y]:.3e} "
           f"layer max |delta| {lm[k, 0]:.3e}")
    print(msg)
    assert worst <= 1.0, msg
