"""C-ABI checks that need no GPU: the library loads, exports every symbol
include/helm.h declares, and rejects invalid arguments before touching the
device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2506_18694_amd import helm
    if not os.path.exists(helm.LIB_PATH):
        pytest.skip("libhelm.so not built")
    return helm, helm.lib()


def test_header_declarations_are_exported():
    helm, L = _lib()
    header = open(os.path.join(ROOT, "include", "helm.h")).read()
    declared = set(re.findall(r"\b(helm_[a-z_0-9]+)\s*\(", header))
    assert declared, "no declarations parsed"
    assert declared == set(helm.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_strerror_and_defaults():
    helm, L = _lib()
    assert helm.strerror(0) == "ok"
    assert "invalid" in helm.strerror(-1)
    o = helm.helm_opts()
    L.helm_opts_default(ctypes.byref(o))
    assert (o.precision, o.nu1, o.nu2, o.hss_m, o.x0_given) == (0, 2, 2, 1, 0)
    assert o.outer == helm.HELM_OUTER_FGMRES
    assert (o.cycle, o.smooth_its) == (helm.HELM_CYCLE_V_JACOBI, 0)
    assert abs(o.omega - 2.0 / 3.0) < 1e-15


def _create(helm, L, dim=2, elem=1, n=8, levels=2, k=5.0, delta=0.0, dh=5.0, opts=None, bc=None):
    mesh = helm.helm_mesh(dim, elem, n, levels)
    out = ctypes.c_void_p(1)
    rc = L.helm_create(ctypes.byref(mesh), k, delta, dh,
                       ctypes.byref(bc) if bc is not None else None,
                       ctypes.byref(opts) if opts is not None else None, None, ctypes.byref(out))
    return rc, out


@pytest.mark.parametrize("kw", [
    dict(dim=4), dict(dim=2, elem=2), dict(dim=3, elem=1), dict(n=1), dict(levels=0),
    dict(n=12, levels=4), dict(k=0.0), dict(k=-1.0), dict(delta=-0.1), dict(dh=0.0),
    dict(delta=2.0, dh=2.0), dict(k=float("nan")), dict(n=128, levels=1),
])
def test_create_rejects_invalid(kw):
    helm, L = _lib()
    rc, out = _create(helm, L, **kw)
    assert rc == helm.HELM_EINVAL
    assert not out.value


def test_create_rejects_bad_options_and_unsupported():
    helm, L = _lib()
    o = helm.helm_opts()
    L.helm_opts_default(ctypes.byref(o))
    o.omega = 2.5
    assert _create(helm, L, opts=o)[0] == helm.HELM_EINVAL
    L.helm_opts_default(ctypes.byref(o))
    o.hss_m = 0
    assert _create(helm, L, opts=o)[0] == helm.HELM_EINVAL
    L.helm_opts_default(ctypes.byref(o))
    o.outer = 2
    assert _create(helm, L, opts=o)[0] == helm.HELM_EINVAL
    L.helm_opts_default(ctypes.byref(o))
    o.cycle = 2
    assert _create(helm, L, opts=o)[0] == helm.HELM_EINVAL
    L.helm_opts_default(ctypes.byref(o))
    o.cycle, o.smooth_its = helm.HELM_CYCLE_W_GMRES, 21
    assert _create(helm, L, opts=o)[0] == helm.HELM_EINVAL
    L.helm_opts_default(ctypes.byref(o))
    o.cycle, o.precision = helm.HELM_CYCLE_W_GMRES, helm.HELM_FP32_MG
    assert _create(helm, L, opts=o)[0] == helm.HELM_ENOTSUP
    # the mixed element: 2D only, V cycles
    assert _create(helm, L, dim=3, elem=helm.HELM_MIXED_DG0_P1)[0] == helm.HELM_EINVAL
    L.helm_opts_default(ctypes.byref(o))
    o.cycle = helm.HELM_CYCLE_W_GMRES
    assert _create(helm, L, elem=helm.HELM_MIXED_DG0_P1, opts=o)[0] == helm.HELM_ENOTSUP
    L.helm_opts_default(ctypes.byref(o))
    o.nu1 = 3
    assert _create(helm, L, opts=o)[0] == helm.HELM_ENOTSUP
    # Dirichlet faces: bits beyond the 2 dim faces, the mixed element, W cycles
    assert _create(helm, L, bc=helm.helm_bc(16))[0] == helm.HELM_EINVAL
    assert _create(helm, L, dim=3, elem=helm.HELM_Q1_HEX, bc=helm.helm_bc(64))[0] == helm.HELM_EINVAL
    assert _create(helm, L, elem=helm.HELM_MIXED_DG0_P1, bc=helm.helm_bc(1))[0] == helm.HELM_ENOTSUP
    L.helm_opts_default(ctypes.byref(o))
    o.cycle = helm.HELM_CYCLE_W_GMRES
    assert _create(helm, L, opts=o, bc=helm.helm_bc(3))[0] == helm.HELM_ENOTSUP
    assert L.helm_create(None, 1.0, 0.0, 1.0, None, None, None, None) == helm.HELM_EINVAL


def test_null_handle_calls_are_rejected():
    helm, L = _lib()
    assert L.helm_destroy(None) == helm.HELM_OK
    assert L.helm_nodes(None, 0) == -1
    assert L.helm_vector_length(None) == -1
    b = ctypes.c_size_t()
    assert L.helm_workspace_bytes(None, 1, ctypes.byref(b)) == helm.HELM_EINVAL
    assert L.helm_solve(None, None, None, 1, 1e-8, None, None) == helm.HELM_EINVAL
    assert L.helm_apply(None, 0, 0, 0, None, None, 1) == helm.HELM_EINVAL
    assert L.helm_vcycle(None, 0, None, None, 1, None) == helm.HELM_EINVAL
    assert L.helm_precondition(None, None, None, 1, None) == helm.HELM_EINVAL
    assert L.helm_hss_history(None, None, None, 1, None, None) == helm.HELM_EINVAL


def test_server_rejects_invalid_options():
    helm, L = _lib()
    out = ctypes.c_void_p(1)
    for o in (helm.helm_server_opts(0.0, 4, 1, 0, 0), helm.helm_server_opts(1e9, 0, 1, 0, 0),
              helm.helm_server_opts(1e9, 4, 7, 0, 0), helm.helm_server_opts(1e9, 4, 1, -1, 0)):
        assert L.helm_server_create(ctypes.byref(o), ctypes.byref(out)) == helm.HELM_EINVAL
    assert L.helm_server_create(None, ctypes.byref(out)) == helm.HELM_EINVAL
    ok = helm.helm_server_opts(1e9, 4, 1, 0, 0)
    assert L.helm_server_create(ctypes.byref(ok), ctypes.byref(out)) == helm.HELM_OK
    rid = ctypes.c_longlong()
    dummy = ctypes.c_void_p(16)
    # nrhs above max_cols, bad mesh, bad tol: rejected before any device work
    assert L.helm_server_submit(out, 2, 64, 4, 6.4, 6.4, dummy, dummy, 5, 1e-8, ctypes.byref(rid)) == helm.HELM_EINVAL
    assert L.helm_server_submit(out, 2, 60, 4, 6.4, 6.4, dummy, dummy, 1, 1e-8, ctypes.byref(rid)) == helm.HELM_EINVAL
    assert L.helm_server_submit(out, 2, 64, 4, 6.4, 6.4, dummy, dummy, 1, 2.0, ctypes.byref(rid)) == helm.HELM_EINVAL
    q, r, b = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
    assert L.helm_server_load(out, ctypes.byref(q), ctypes.byref(r), ctypes.byref(b)) == helm.HELM_OK
    assert (q.value, r.value, b.value) == (0, 0, 0.0)
    assert L.helm_server_destroy(out) == helm.HELM_OK


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """No CPU fallback: with libhelm.so absent, loading the binding raises
    and a solver cannot be created."""
    from paper_2506_18694_amd import helm
    monkeypatch.setattr(helm, "_lib", None)
    monkeypatch.setattr(helm, "LIB_PATH", str(tmp_path / "libhelm.so"))
    with pytest.raises(ImportError):
        helm.lib()
    with pytest.raises(ImportError):
        helm.Solver(2, 8, 2, 2.0, 0.0, 2.0)
