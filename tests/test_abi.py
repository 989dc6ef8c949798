"""CPU checks of the C ABI: the library loads, exports every function declared in
include/cgks.h, and rejects bad arguments on the host before any device work."""
import ctypes as C
import os
import re

import pytest

from paper_2508_08965_amd import cgks as K

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "cgks.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cgks_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_path():
    names = declared_functions()
    for must in ["cgks_ctx_create", "cgks_ctx_destroy", "cgks_dt", "cgks_stage", "cgks_step", "cgks_check"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(K.LIB_PATH):
        pytest.skip("library not built")
    lib = C.CDLL(K.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_host_side_argument_errors():
    if not os.path.exists(K.LIB_PATH):
        pytest.skip("library not built")
    L = K.lib()
    p = K.default_params()
    h = C.c_void_p()
    dims = (C.c_int * 3)(4, 4, 4)
    nodes = (C.POINTER(C.c_double) * 1)()
    # no blocks / NULL node pointer / bad parameters: all rejected before touching the device
    assert L.cgks_ctx_create(C.byref(h), 0, dims, nodes, C.byref(p), None) == K.EINVAL
    assert L.cgks_ctx_create(C.byref(h), 1, dims, nodes, C.byref(p), None) == K.EINVAL
    bad = K.default_params(gamma=0.9)
    assert L.cgks_ctx_create(C.byref(h), 1, dims, nodes, C.byref(bad), None) == K.EINVAL
    bad = K.default_params(viscous=1, mu0=0.0)
    assert L.cgks_ctx_create(C.byref(h), 1, dims, nodes, C.byref(bad), None) == K.EINVAL
    bad = K.default_params(recon_prec=7)
    assert L.cgks_ctx_create(C.byref(h), 1, dims, nodes, C.byref(bad), None) in (K.EINVAL, K.EUNSUPPORTED)
    assert K.last_error() != ""
    assert L.cgks_stage(None, 1, None, None, None, None, None) == K.EINVAL
    assert L.cgks_step(None, None, None, None, None, 1, None) == K.EINVAL
    f = C.c_int()
    assert L.cgks_check(None, C.byref(f)) == K.EINVAL
    assert L.cgks_num_cells(None) == 0
    bad = K.default_params(per_block=2)
    assert L.cgks_ctx_create(C.byref(h), 1, dims, nodes, C.byref(bad), None) == K.EINVAL
    # per-cell stored matrices: FP64 only; no fourth implementation
    bad = K.default_params(recon_impl=3)
    assert L.cgks_ctx_create(C.byref(h), 1, dims, nodes, C.byref(bad), None) == K.EINVAL
    for kw in (dict(recon_prec=2), dict(recon_prec=1), dict(flux_prec=1)):
        bad = K.default_params(recon_impl=2, **kw)
        assert L.cgks_ctx_create(C.byref(h), 1, dims, nodes, C.byref(bad), None) == K.EUNSUPPORTED
    cfg = K.Launch(128, 0, 0)
    assert L.cgks_get_launch(None, 1, C.byref(cfg)) == K.EINVAL
    assert L.cgks_set_launch(None, 1, C.byref(cfg)) == K.EINVAL
    assert L.cgks_autotune(None, None, None, None, None, 1, None, 0, None) == K.EINVAL
    assert L.cgks_step_graph(None, None, None, None, None, 1, None) == K.EINVAL
    assert L.cgks_diagnostics(None, None, None, None, None) == K.EINVAL


def test_default_params_are_the_papers_constants():
    if not os.path.exists(K.LIB_PATH):
        pytest.skip("library not built")
    p = K.default_params()
    assert p.gamma == 1.4 and p.cfl == 0.5 and p.tau_eps == 0.05 and p.tau_C == 5.0
    assert p.geno_eps == 1e-15 and p.geno_r == 2.0


def test_wall_sides_rejected_on_the_host():
    """Side types and wall geometry are checked before the device is touched."""
    if not os.path.exists(K.LIB_PATH):
        pytest.skip("library not built")
    import numpy as np
    from paper_2508_08965_amd import workloads as W
    L = K.lib()
    h = C.c_void_p()
    dims = (C.c_int * 3)(4, 4, 4)

    def create(nodes, **kw):
        a = np.ascontiguousarray(nodes.numpy(), dtype=np.float64)
        ptrs = (C.POINTER(C.c_double) * 1)(a.ctypes.data_as(C.POINTER(C.c_double)))
        return L.cgks_ctx_create(C.byref(h), 1, dims, ptrs, C.byref(K.default_params(**kw)), None)

    box = W.cartesian_nodes((4, 4, 4))
    for bc in ((1, 0, 0, 0, 0, 0), (0, 0, 2, 0, 0, 0), (4, 4, 0, 0, 0, 0), (-1, -1, 0, 0, 0, 0)):
        assert create(box, bc=bc) == K.EINVAL, bc
    assert create(box, bc=(1, 1, 0, 0, 0, 0), recon_impl=1) == K.EUNSUPPORTED
    # sides that are planes but not normal to their axis
    assert create(W.skewed_nodes((4, 4, 4)), bc=(1, 1, 0, 0, 0, 0)) == K.EINVAL
    # x sides whose tangential node coordinates differ (one side moved in y)
    moved = box.clone()
    moved[:, :, 4, 1] += 0.01
    assert create(moved, bc=(1, 1, 0, 0, 0, 0)) == K.EINVAL
    assert "wall side" in K.last_error()


def test_far_field_state_checked_on_the_host():
    if not os.path.exists(K.LIB_PATH):
        pytest.skip("library not built")
    import numpy as np
    from paper_2508_08965_amd import workloads as W
    L = K.lib()
    h = C.c_void_p()
    dims = (C.c_int * 3)(4, 4, 4)
    a = np.ascontiguousarray(W.cartesian_nodes((4, 4, 4)).numpy())
    ptrs = (C.POINTER(C.c_double) * 1)(a.ctypes.data_as(C.POINTER(C.c_double)))
    for far in ((0.0, 0, 0, 0, 2.5), (1.0, 0, 0, 0, 0.0), (1.0, 3.0, 0, 0, 2.5)):  # rho 0, p 0, p < 0
        p = K.default_params(bc=(3, 3, 0, 0, 0, 0), farfield=far)
        assert L.cgks_ctx_create(C.byref(h), 1, dims, ptrs, C.byref(p), None) == K.EINVAL, far
    p = K.default_params(bc=(4, 4, 0, 0, 0, 0))
    assert L.cgks_ctx_create(C.byref(h), 1, dims, ptrs, C.byref(p), None) == K.EINVAL
