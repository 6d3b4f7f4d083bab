"""Host-side checks of the C ABI library (no GPU needed): it loads, exports
every function include/xod.h declares, and rejects invalid descriptions
before touching the device."""

import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2512_06729_amd", "libxod.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libxod.so not built")


def test_library_exports_every_header_symbol():
    import paper_2512_06729_amd as xod
    syms = xod.header_symbols()
    assert len(syms) >= 20
    lib = ctypes.CDLL(LIB)
    missing = [s for s in syms if not hasattr(lib, s)]
    assert missing == []


def test_header_is_plain_c(tmp_path):
    """include/xod.h compiles as C99 with every warning an error, and each
    declared entry point is a file-scope function of that name."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    import paper_2512_06729_amd as xod
    src = tmp_path / "h.c"
    calls = "\n".join(f"  (void)&{s};" for s in xod.header_symbols())
    src.write_text('#include "xod.h"\nint main(void) {\n' + calls + "\n  return 0;\n}\n")
    r = subprocess.run([cc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                        "-I", os.path.join(ROOT, "include"), "-c", str(src), "-o",
                        str(tmp_path / "h.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_binding_covers_every_header_symbol():
    """Each entry point of include/xod.h has a typed binding (the status
    calls in the signature table; the workspace-size query, which returns a
    size, directly), and nothing is bound that the header does not declare."""
    import paper_2512_06729_amd as xod
    declared = set(xod.header_symbols())
    bound = set(xod._f)
    assert declared - bound == {"xod_photolysis_workspace"}
    assert bound <= declared
    assert xod.photolysis_workspace(1, 1, 1, 1) > 0


def _desc(xod, S=3, reac=None):
    keep = dict(comp=np.ones((1, S), np.int32), mass=np.full(S, 10.0),
                nasa=np.zeros((S, 2, 7)), rtype=np.zeros(1, np.int32),
                reac=np.array(reac if reac is not None else [[0, 1, -1]], np.int32),
                prod=np.array([[2, -1, -1]], np.int32), rev=np.ones(1, np.int32),
                kooij=np.zeros(1, np.int32), params=np.zeros((1, 6)))
    p = xod._ptr
    d = xod.NetworkDesc(S, 1, 1, p(keep["comp"], ctypes.c_int32), p(keep["mass"], ctypes.c_double),
                        p(keep["nasa"], ctypes.c_double), 1000.0, p(keep["rtype"], ctypes.c_int32),
                        p(keep["reac"], ctypes.c_int32), p(keep["prod"], ctypes.c_int32),
                        p(keep["rev"], ctypes.c_int32), p(keep["kooij"], ctypes.c_int32),
                        p(keep["params"], ctypes.c_double))
    return d, keep


@pytest.mark.parametrize("reac,msg", [([[0, 7, -1]], "out of range"),
                                      ([[-1, -1, -1]], "without reactant")])
def test_network_create_rejects_bad_descriptions(reac, msg):
    import paper_2512_06729_amd as xod
    d, keep = _desc(xod, reac=reac)
    h = ctypes.c_void_p()
    st = xod._f["xod_network_create"](ctypes.byref(d), ctypes.byref(h))
    assert st == xod.XOD_EINVAL
    assert msg in xod.last_error()
    assert not h.value


def test_null_arguments_are_einval():
    import paper_2512_06729_amd as xod
    assert xod._f["xod_network_create"](None, None) == xod.XOD_EINVAL
    assert xod._f["xod_step"](None, 1.0, None) == xod.XOD_EINVAL
    assert xod._f["xod_step_frozen"](None, 1.0, None) == xod.XOD_EINVAL
    assert xod._f["xod_step_ros2"](None, 1.0, None) == xod.XOD_EINVAL
    assert xod._f["xod_step_bdf2"](None, 1.0, None) == xod.XOD_EINVAL
    assert xod._f["xod_step_newton"](None, 1.0, 2, None) == xod.XOD_EINVAL
    assert xod._f["xod_column_set_boundary"](None, None) == xod.XOD_EINVAL
    assert xod._f["xod_column_destroy"](None) == xod.XOD_EINVAL
    assert xod._f["xod_set_option"](b"nope", 1) == xod.XOD_EINVAL
    assert xod._f["xod_set_option"](b"gemm", 3) == xod.XOD_EINVAL
    buf = ctypes.create_string_buffer(8)
    assert xod._f["xod_last_error"](buf, 8) == xod.XOD_OK
    assert len(buf.value) <= 7


def test_photolysis_entry_validates_before_any_launch():
    """Size, mu and workspace checks of xod_photolysis_spectral need no GPU."""
    import ctypes
    import paper_2512_06729_amd as xod
    f = xod._f["xod_photolysis_spectral"]
    fake = ctypes.c_void_p(16)
    assert xod.photolysis_workspace(0, 1, 1, 1) == 0
    assert xod.photolysis_workspace(150, 463, 10000, 772) > 8 * 150 * 10000
    args = dict(N=2, S=2, A=1, L=3, P=1)
    def call(N=2, S=2, A=1, L=3, P=1, mu=1.0, work=fake, nbytes=1 << 30):
        return f(N, S, A, L, P, fake, fake, fake, fake, fake, fake, fake, 1.0, mu, work, nbytes,
                 fake, None)
    assert call(N=0) == xod.XOD_EINVAL
    assert call(L=0) == xod.XOD_EINVAL
    assert call(A=-1) == xod.XOD_EINVAL
    assert call(mu=0.0) == xod.XOD_EINVAL
    assert call(work=None) == xod.XOD_EINVAL
    assert call(nbytes=8) == xod.XOD_EINVAL
    assert "workspace" in xod.last_error()
    del args
