"""Host-side checks of the C ABI that need no GPU: every function declared in
include/*.h is exported by libfd.so, and argument / stability errors are
reported before any device is touched."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(fd\w*|nn\w*)\s*\(", txt, re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2312_13094_amd import fd, build
    if not os.path.exists(fd.LIB_PATH):
        build.build()
    return fd.lib()


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["fd_create_grid", "fd_forward", "fd_adjoint", "fd_pack_halo", "fd_unpack_halo",
                 "fd_destroy_grid", "fd_last_error", "fd_sparse_prepare", "fd_set_model"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def _desc(fd, **kw):
    d = fd.GridDesc()
    d.ndim = kw.get("ndim", 3)
    for k, s in enumerate(kw.get("shape", (32, 32, 32))):
        d.shape[k] = s
        d.spacing[k] = 10.0
    d.space_order = kw.get("so", 8)
    d.nbl = kw.get("nbl", 4)
    d.physics = kw.get("physics", 0)
    d.boundary = kw.get("boundary", 0)
    d.dt = kw.get("dt", 5e-4)
    d.vmax = kw.get("vmax", 4500.0)
    d.device = 0
    return d


def test_cfl_violation_is_unstable(lib):
    from paper_2312_13094_amd import fd, synth
    h = ctypes.c_void_p()
    lim = synth.courant_limit(8, 3) * 10.0 / 4500.0
    rc = lib.fd_create_grid(ctypes.byref(_desc(fd, dt=lim * 1.01)), ctypes.byref(h))
    assert rc == fd.FD_EUNSTABLE
    assert b"stability" in lib.fd_last_error()


@pytest.mark.parametrize("kw", [dict(so=7), dict(so=18), dict(ndim=4), dict(nbl=40, shape=(32, 32, 32)),
                                dict(shape=(1, 32, 32)), dict(boundary=5), dict(dt=0.0)])
def test_bad_descriptor_is_einval(lib, kw):
    from paper_2312_13094_amd import fd
    h = ctypes.c_void_p()
    rc = lib.fd_create_grid(ctypes.byref(_desc(fd, **kw)), ctypes.byref(h))
    assert rc == fd.FD_EINVAL


def test_null_arguments(lib):
    from paper_2312_13094_amd import fd
    assert lib.fd_create_grid(None, None) == fd.FD_EINVAL
    assert lib.fd_forward(None, None, None, None, None, None, 0, None, 0, None) == fd.FD_EINVAL
    assert lib.fd_pack_halo(None, None, 0, None, None) == fd.FD_EINVAL
    assert lib.fd_halo_face_elems(None, 0) < 0
    assert lib.fd_step(None, None, None, None, None, None, None, None) == fd.FD_EINVAL
    assert lib.fd_step_lagged(None, None, None, None, None, None, None, None) == fd.FD_EINVAL


def test_network_entry_points_reject_bad_arguments():
    """Shape and pointer checks of the network calls return FD_EINVAL before
    any launch (so they run without a GPU)."""
    from paper_2312_13094_amd import fd, nn
    L = nn.lib()
    v = nn.View(0, 1, 1)
    x = ctypes.c_void_p(16)
    # empty volume, then a missing field pointer
    assert L.nn_conv_gelu_fields(0, 4, 4, x, v, x, v, x, v, 1, None, x, x, None, x,
                                 None) == fd.FD_EINVAL
    assert L.nn_conv_gelu_fields(4, 4, 4, None, v, x, v, x, v, 1, None, x, x, None, x,
                                 None) == fd.FD_EINVAL
    assert b"nn_conv_gelu_fields" in lib_error(L)
    assert L.nn_conv_gelu(3, 4, 4, 4, x, x, x, None, x, None) == fd.FD_EINVAL
    assert L.nn_rms(4, 4, 4, None, v, x, None, None) == fd.FD_EINVAL


def lib_error(L):
    return L.fd_last_error()


def test_binding_rejects_short_pointer_arrays():
    """The library reads a fixed number of device pointers from an array
    argument (per physics and call); the binding refuses a shorter list
    before the call, so no stray address can reach a kernel."""
    from paper_2312_13094_amd import fd
    with pytest.raises(fd.FdError) as e:
        fd._ptr_array([None] * 4, 5, "set_model")
    assert e.value.code == fd.FD_EINVAL
    assert fd._ptr_array([None] * 5, 5) is not None
    assert fd._ptr_array(None, 5) is None
    assert fd.Grid._AUX == {fd.FD_ACOUSTIC: 0, fd.FD_TTI: 4, fd.FD_ELASTIC: 2, fd.FD_VISCO: 5}
    assert fd.Grid._NSTATE == {fd.FD_ACOUSTIC: 2, fd.FD_TTI: 4, fd.FD_ELASTIC: 9,
                               fd.FD_VISCO: 15}
