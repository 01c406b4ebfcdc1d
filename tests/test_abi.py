"""C-ABI checks that need no GPU: the shared library loads, exports every
function that include/boxscreen.h declares, and rejects bad arguments before
touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2202_07258_amd import native as N

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "boxscreen.h")


def _declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z_0-9]*\s*\*?\s*([A-Za-z_][A-Za-z_0-9]*)\s*\(",
                       txt, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(N.LIBRARY_PATH):
        pytest.fail("libboxscreen.so not built: run python -m paper_2202_07258_amd.build")
    return N.load()


def test_header_declares_expected_entry_points():
    names = _declared_functions()
    for n in ["solve_bvls", "solve_nnls", "solve_bvls_varbatch", "bxs_last_error", "bxs_version",
              "bxs_default_opts", "bxs_workspace_size", "bxs_workspace_size_batch"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert sorted(N.EXPORTED) == sorted(_declared_functions())


def test_default_opts(lib):
    o = N.Opts()
    lib.bxs_default_opts(C.byref(o))
    assert (o.solver, o.screening, o.screen_every, o.max_iter, o.eps_gap, o.step, o.power_iters) == \
        (0, 1, 10, 100000, 1e-6, 0.0, 0)
    assert not o.t and not o.workspace and not o.stream
    assert o.fidelity == 0 and o.deterministic in (0, 1)      # least squares; reductions always fixed-order


def _opts(lib, **kw):
    o = N.Opts()
    lib.bxs_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


FAKE = 1 << 20   # never dereferenced: every case below fails validation first


@pytest.mark.parametrize("m,n,lda,code", [(0, 5, 1, N.BXS_ERR_SHAPE), (5, 0, 5, N.BXS_ERR_SHAPE),
                                          (5, 5, 4, N.BXS_ERR_SHAPE), (20000, 5, 20000, N.BXS_ERR_SHAPE),
                                          (N.MAX_ROWS + 1, 5, N.MAX_ROWS + 1, N.BXS_ERR_SHAPE)])
def test_shape_errors(lib, m, n, lda, code):
    o = _opts(lib)
    info = N.Info()
    st = lib.solve_bvls(m, n, 0, FAKE, lda, FAKE, FAKE, FAKE, FAKE, FAKE, C.byref(o), C.byref(info))
    assert st == code
    assert lib.bxs_last_error().decode()


@pytest.mark.parametrize("field,value", [("solver", 7), ("screening", 2), ("screen_every", 0),
                                         ("max_iter", 0), ("eps_gap", -1.0), ("eps_gap", float("inf")),
                                         ("step", float("nan")), ("fidelity", 2), ("fidelity", 1),
                                         ("deterministic", 2)])
def test_option_errors(lib, field, value):
    o = _opts(lib, **{field: value})
    st = lib.solve_nnls(8, 8, 0, FAKE, 8, FAKE, FAKE, FAKE, C.byref(o), None)
    assert st == N.BXS_ERR_ARG


@pytest.mark.parametrize("kw", [dict(huber_delta=0.0), dict(huber_delta=-1.0), dict(huber_delta=float("inf")),
                                dict(huber_delta=float("nan")), dict(huber_delta=1.0, solver=N.BXS_CD),
                                dict(huber_delta=1.0, theta_star=FAKE)])
def test_huber_option_errors(lib, kw):
    # the Huber fidelity needs a finite delta > 0, the PG or CP solver and no theta*
    o = _opts(lib, fidelity=1, **kw)
    assert lib.solve_nnls(8, 8, 0, FAKE, 8, FAKE, FAKE, FAKE, C.byref(o), None) == N.BXS_ERR_ARG
    assert lib.bxs_last_error().decode()


def test_huber_rejected_by_shared_matrix_solver_and_adjoint(lib):
    o = _opts(lib, fidelity=1, huber_delta=1.0)
    assert lib.solve_nnls_batched_shared(8, 8, 2, 0, FAKE, 8, FAKE, 8, FAKE, 8, FAKE, 8, C.byref(o), None) \
        == N.BXS_ERR_ARG
    assert "least squares" in lib.bxs_last_error().decode()
    assert lib.nnls_adjoint(8, 8, 2, 0, FAKE, 8, FAKE, 8, FAKE, 8, FAKE, 8, FAKE, 8, None, 8, None, 8,
                            C.byref(o), None) == N.BXS_ERR_ARG
    assert "least-squares" in lib.bxs_last_error().decode()


def test_cd_block_switch_and_workspace(lib):
    # the switch takes 0 or 1; the block form's workspace adds its Gram and
    # cross blocks (2 x 128 doubles per column), the one-workgroup form does not
    assert lib.bxs_set_cd_block(2) == N.BXS_ERR_ARG
    o = _opts(lib, solver=N.BXS_CD)
    sizes = []
    for enable in (1, 0):
        assert lib.bxs_set_cd_block(enable) == N.BXS_OK
        b = C.c_size_t(0)
        assert lib.bxs_workspace_size(2000, 6000, C.byref(o), C.byref(b)) == N.BXS_OK
        sizes.append(b.value)
    assert lib.bxs_set_cd_block(1) == N.BXS_OK
    assert sizes[0] - sizes[1] >= 2 * 128 * 8 * 6000


def test_normal_equations_direction_needs_tall_matrix(lib):
    o = _opts(lib, t_choice=N.T_CHOICES["normal_equations"])
    assert lib.solve_nnls(8, 16, 0, FAKE, 8, FAKE, FAKE, FAKE, C.byref(o), None) == N.BXS_ERR_ARG
    assert "n <= m" in lib.bxs_last_error().decode()


def test_null_arguments(lib):
    o = _opts(lib)
    assert lib.solve_bvls(8, 8, 0, None, 8, FAKE, FAKE, FAKE, FAKE, FAKE, C.byref(o), None) == N.BXS_ERR_ARG
    assert lib.solve_bvls(8, 8, 0, FAKE, 8, FAKE, None, FAKE, FAKE, FAKE, C.byref(o), None) == N.BXS_ERR_ARG
    assert lib.solve_nnls(8, 8, 0, FAKE, 8, FAKE, FAKE, FAKE, None, None) == N.BXS_ERR_ARG
    assert lib.solve_nnls(8, 8, 5, FAKE, 8, FAKE, FAKE, FAKE, C.byref(o), None) == N.BXS_ERR_ARG
    assert lib.solve_bvls_varbatch(0, 0, None, C.byref(o), None) == N.BXS_ERR_ARG


def test_group_scale_setter(lib):
    assert lib.bxs_set_group_scale(0, 0.001) == N.BXS_ERR_ARG
    assert lib.bxs_set_group_scale(0, 5.0) == N.BXS_ERR_ARG
    assert lib.bxs_set_group_scale(99, 1.0) == N.BXS_ERR_ARG
    assert lib.bxs_group_scale(99) == 0.0
    assert lib.bxs_set_group_scale(3, 0.25) == N.BXS_OK and lib.bxs_group_scale(3) == 0.25
    assert lib.bxs_set_group_scale(3, 1.0) == N.BXS_OK and lib.bxs_group_scale(3) == 1.0


def test_workspace_query_row_limit(lib):
    o = N.Opts()
    lib.bxs_default_opts(C.byref(o))
    b = C.c_size_t(0)
    assert lib.bxs_workspace_size(N.MAX_ROWS, 10, C.byref(o), C.byref(b)) == N.BXS_OK and b.value > 0
    assert lib.bxs_workspace_size(N.MAX_ROWS + 1, 10, C.byref(o), C.byref(b)) == N.BXS_ERR_SHAPE


def test_step_estimate_option(lib):
    """power_iters: at most 64 Lanczos steps; their workspace (two m-vectors and
    the tridiagonal coefficients) is only reserved when the step is computed."""
    o = N.Opts()
    lib.bxs_default_opts(C.byref(o))
    b8, b64, bstep = C.c_size_t(0), C.c_size_t(0), C.c_size_t(0)
    assert lib.bxs_workspace_size(1000, 50, C.byref(o), C.byref(b8)) == N.BXS_OK
    o.power_iters = 64
    assert lib.bxs_workspace_size(1000, 50, C.byref(o), C.byref(b64)) == N.BXS_OK
    assert b64.value >= b8.value
    o.power_iters = 65
    assert lib.bxs_workspace_size(1000, 50, C.byref(o), C.byref(b64)) == N.BXS_ERR_ARG
    o.power_iters = 0
    o.step = 0.1
    assert lib.bxs_workspace_size(1000, 50, C.byref(o), C.byref(bstep)) == N.BXS_OK
    assert bstep.value < b8.value


def test_workspace_query_shape_check(lib):
    o = _opts(lib)
    b = C.c_size_t(0)
    assert lib.bxs_workspace_size(0, 10, C.byref(o), C.byref(b)) == N.BXS_ERR_SHAPE


def test_batched_argument_errors(lib):
    o = _opts(lib)
    f = lib.solve_nnls_batched_shared
    assert f(0, 5, 3, 0, FAKE, 1, FAKE, 1, FAKE, 5, FAKE, 5, C.byref(o), None) == N.BXS_ERR_SHAPE
    assert f(5, 5, 3, 0, FAKE, 4, FAKE, 5, FAKE, 5, FAKE, 5, C.byref(o), None) == N.BXS_ERR_SHAPE
    assert f(5, 5, 3, 0, None, 5, FAKE, 5, FAKE, 5, FAKE, 5, C.byref(o), None) == N.BXS_ERR_ARG
    o2 = _opts(lib, iter_precision=9)
    assert f(5, 5, 3, 0, FAKE, 5, FAKE, 5, FAKE, 5, FAKE, 5, C.byref(o2), None) == N.BXS_ERR_ARG
    o3 = _opts(lib, solver=1)
    assert f(5, 5, 3, 0, FAKE, 5, FAKE, 5, FAKE, 5, FAKE, 5, C.byref(o3), None) == N.BXS_ERR_ARG
