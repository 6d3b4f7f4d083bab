"""The allocation-free spectral photolysis entry point
(xod_photolysis_spectral_noalloc: the workspace is the library's fixed
device array) against the entry point with a caller's workspace
(xod_photolysis_spectral), through the C ABI: two calls in a row, the second
with a smaller input, each compared with the workspace entry point on the
same inputs (the same kernels on the same data: the bits must agree), plus
the oracle on the second; and the size limit refused on the host."""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import synth  # noqa: E402
from oracle import grid as grid_mod, photolysis as ph  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm device")
    import paper_2512_06729_amd  # noqa: F401  (fails loudly if not built)


def device_args(n, dz, absorbers, sig_ext, J0, dlam, sig_ph):
    dev = torch.device("cuda:0")
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a), device=dev)   # noqa: E731
    A, L = len(absorbers), len(J0)
    return (d(n), d(dz), d(np.asarray(absorbers, np.int32)), d(np.reshape(sig_ext, (A, L))),
            d(J0), d(dlam), d(sig_ph))


def both(args, t_f, mu):
    import paper_2512_06729_amd as xod
    n, dz, ab, se, J0, dl, sph = args
    N, A, L, P = n.shape[0], ab.shape[0], J0.shape[0], sph.shape[0]
    stream = torch.cuda.current_stream().cuda_stream
    k_ws = torch.full((N, P), np.nan, dtype=torch.float64, device=n.device)
    k_na = torch.full((N, P), np.nan, dtype=torch.float64, device=n.device)
    work = torch.empty(xod.photolysis_workspace(N, A, L, P), dtype=torch.uint8, device=n.device)
    xod.photolysis_spectral(n, dz, ab, se, J0, dl, sph, k_ws, work, t_f=t_f, mu=mu,
                            stream=stream)
    xod.photolysis_spectral_noalloc(n, dz, ab, se, J0, dl, sph, k_na, t_f=t_f, mu=mu,
                                    stream=stream)
    torch.cuda.synchronize()
    return k_ws.cpu().numpy(), k_na.cpu().numpy()


def test_noalloc_matches_workspace_entry_point_twice():
    net, col = synth.make_config(3)
    sp = synth.make_spectrum(net)
    dz = grid_mod.make_grid(col, net.mass_amu).dz
    # first call: the full 594-species workload (150 layers, 10,000 bins)
    print("no-alloc photolysis: call 1, 150 x 10000 bins, 463 absorbers", flush=True)
    full = (col.n0, dz, sp["absorbers"], sp["sig_ext"], sp["J0"], sp["dlam"], sp["sig_ph"])
    ws, na = both(device_args(*full), 0.5, 0.7)
    assert np.all(np.isfinite(na))
    np.testing.assert_array_equal(na, ws)
    # second call, smaller in every dimension: the array keeps the first
    # call's contents, none of which may leak into this result
    print("no-alloc photolysis: call 2, 37 x 1500 bins, 40 absorbers", flush=True)
    N2, L2, A2, P2 = 37, 1500, 40, 129
    L = len(sp["J0"])
    sig_ext = np.reshape(sp["sig_ext"], (-1, L))[:A2, :L2]
    small = (col.n0[-N2:], dz[-N2:], sp["absorbers"][:A2], sig_ext, sp["J0"][:L2],
             sp["dlam"][:L2], sp["sig_ph"][:P2, :L2])
    ws2, na2 = both(device_args(*small), 1.0, 1.0)
    np.testing.assert_array_equal(na2, ws2)
    o = ph.spectral_rates(*small, t_f=1.0, mu=1.0)
    scale = np.abs(o).max(axis=0, keepdims=True)
    assert np.all(np.abs(na2 - o) <= 1e-11 * np.abs(o) + 1e-12 * scale)


def test_noalloc_refuses_sizes_beyond_its_array():
    import paper_2512_06729_amd as xod
    N, A, L, P = 150, 463, 40000, 772
    assert xod.photolysis_workspace(N, A, L, P) > 64 << 20
    dev = torch.device("cuda:0")
    n = torch.zeros((N, 594), dtype=torch.float64, device=dev)
    dz = torch.ones(N, dtype=torch.float64, device=dev)
    ab = torch.zeros(A, dtype=torch.int32, device=dev)
    se = torch.zeros((A, L), dtype=torch.float64, device=dev)
    J0 = torch.zeros(L, dtype=torch.float64, device=dev)
    sph = torch.zeros((P, L), dtype=torch.float64, device=dev)
    kph = torch.zeros((N, P), dtype=torch.float64, device=dev)
    with pytest.raises(xod.XodError) as e:
        xod.photolysis_spectral_noalloc(n, dz, ab, se, J0, J0, sph, kph)
    assert e.value.status == xod.XOD_EINVAL
    assert "workspace" in str(e.value)
