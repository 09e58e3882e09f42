"""C ABI checks that need no GPU: the library loads, exports every declared symbol, and
rejects bad arguments with the documented codes before touching the device."""
import ctypes
import glob
import math
import os
import re

import numpy as np
import pytest

from paper_1701_02011_amd import _lib
from paper_1701_02011_amd.synth import make_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="session")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1701_02011_amd import _build
        _build.build()
    return _lib.load()


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(dsrg_\w+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "dsrg_pt2_energy" in names and "dsrg_pt3_energy" in names
    for n in names:
        assert hasattr(lib, n), n
    assert lib.dsrg_version() >= 100
    assert lib.dsrg_release_cache() == 0


def _call(p, mutate=None, opt=None):
    keep = []
    st, fl = _lib._problem_struct(p, keep)
    if mutate:
        mutate(st)
    r = _lib.Result()
    r.e2 = 12345.0
    o = opt or _lib.Options(fl, 0, 0, None)
    rc = _lib.load().dsrg_pt3_energy(ctypes.byref(st), ctypes.byref(o), ctypes.byref(r))
    return rc, r


@pytest.mark.parametrize("mut,code", [
    (lambda s: setattr(s, "n_core", -1), _lib.DSRG_E_ARG),
    (lambda s: setattr(s, "n_aux", 0), _lib.DSRG_E_ARG),
    (lambda s: setattr(s, "s", 0.0), _lib.DSRG_E_ARG),
    (lambda s: setattr(s, "s", -1.0), _lib.DSRG_E_ARG),
    (lambda s: setattr(s, "s", float("nan")), _lib.DSRG_E_ARG),
    (lambda s: setattr(s, "B", None), _lib.DSRG_E_ARG),
    (lambda s: setattr(s, "gamma1", None), _lib.DSRG_E_ARG),
])
def test_bad_arguments(lib, mut, code):
    p = make_problem(1, 2, 3, 6, seed=1)
    rc, r = _call(p, mut)
    assert rc == code
    assert r.e2 == 12345.0               # output untouched
    assert len(lib.dsrg_last_error()) > 0


def test_non_finite_input(lib):
    p = make_problem(1, 2, 3, 6, seed=1)
    p.B[2, 1, 3] = np.nan
    rc, r = _call(p)
    assert rc == _lib.DSRG_E_NONFINITE and r.e2 == 12345.0
    p = make_problem(1, 2, 3, 6, seed=1)
    p.gamma2[1, 0, 0, 0, 0] = np.inf
    rc, _ = _call(p)
    assert rc == _lib.DSRG_E_NONFINITE


def test_unsupported_options(lib):
    p = make_problem(1, 2, 3, 6, seed=1)
    for precision in (3, -1, 7):
        rc, _ = _call(p, opt=_lib.Options(0, precision, 0, None))
        assert rc == _lib.DSRG_E_UNSUPPORTED
    # 17 active orbitals: above the largest active space built (16)
    import dataclasses
    n = 18
    p = dataclasses.replace(make_problem(0, 2, 1, 4, seed=1), n_active=17, eps=np.zeros(n),
                            B=np.zeros((4, n, n)), gamma1=np.zeros((2, 17, 17)),
                            gamma2=np.zeros((3,) + (17,) * 4), gamma3=None, f_offdiag=None)
    rc, _ = _call(p)
    assert rc == _lib.DSRG_E_UNSUPPORTED


def test_null_problem(lib):
    r = _lib.Result()
    rc = lib.dsrg_pt3_energy(None, None, ctypes.byref(r))
    assert rc == _lib.DSRG_E_ARG


def test_batch_rejects_bad_items_without_gpu(lib):
    """Every item fails validation on the host: the call returns the first item's code."""
    p = make_problem(1, 2, 3, 6, seed=1)
    keep = []
    st, fl = _lib._problem_struct(p, keep)
    st.n_aux = 0
    st2, _ = _lib._problem_struct(p, keep)
    st2.s = -1.0
    arr = (_lib.Problem * 2)(st, st2)
    res = (_lib.Result * 2)()
    status = (ctypes.c_int32 * 2)()
    rc = lib.dsrg_pt3_energy_batch(arr, 2, None, res, status)
    assert rc == _lib.DSRG_E_ARG and list(status) == [_lib.DSRG_E_ARG, _lib.DSRG_E_ARG]
    assert lib.dsrg_pt3_energy_batch(arr, 0, None, res, status) == _lib.DSRG_E_ARG


def test_test_gett_validates_strides(lib):
    A = np.zeros(4); B = np.zeros(4); C = np.zeros(4)
    with pytest.raises(_lib.DsrgError) as e:
        _lib.test_gett(A, B, C, m=[(3, 2, 1)], n=[(2, 1, 1)], k=[(2, 1, 2)])
    assert e.value.code == _lib.DSRG_E_ARG
    A = np.zeros(4); B = np.zeros(4); C = np.zeros(4)
    with pytest.raises(_lib.DsrgError) as e:
        _lib.test_gett(A, B, C, m=[(2, 1, 1)], n=[(2, 1, 2)], k=[(2, 2, 1)], precision=5)
    assert e.value.code == _lib.DSRG_E_UNSUPPORTED


def _opt(flags=0, precision=0, cap=0, virt_batch=0):
    return _lib.Options(flags, precision, cap, None, virt_batch)


def test_density_checks(lib):
    """gamma1 must be symmetric, gamma2 Hermitian and antisymmetric in its same-spin blocks
    (DSRG_E_RDM, output untouched)."""
    p = make_problem(1, 3, 2, 6, seed=1)
    assert _call(p)[0] != _lib.DSRG_E_RDM   # valid densities pass the host checks
    q = make_problem(1, 3, 2, 6, seed=1)
    q.gamma1[1, 0, 2] += 1e-6
    rc, r = _call(q)
    assert rc == _lib.DSRG_E_RDM and r.e2 == 12345.0
    q = make_problem(1, 3, 2, 6, seed=1)
    q.gamma2[0, 0, 1, 0, 2] += 1e-6      # aa block: breaks u <-> v antisymmetry
    assert _call(q)[0] == _lib.DSRG_E_RDM
    q = make_problem(1, 3, 2, 6, seed=1)
    q.gamma2[1, 0, 1, 2, 0] += 1e-6      # ab block: breaks hermiticity only
    assert _call(q)[0] == _lib.DSRG_E_RDM
    q = make_problem(1, 3, 2, 6, seed=1)
    q.gamma2[1, 0, 1, 2, 0] += 1e-12     # below the tolerance
    assert _call(q)[0] != _lib.DSRG_E_RDM


def test_intruder_at_infinite_s(lib):
    """s = +inf with a vanishing singles or doubles denominator: DSRG_E_INTRUDER; the same
    orbital energies at finite s are accepted (the regulariser has no intruders)."""
    p = make_problem(2, 0, 3, 6, seed=1, s=float("inf"))
    p.eps[:] = [-1.0, -0.5, 0.25, 0.75, 2.0]      # e0 + e1 = -1.5: no zero denominator
    assert _call(p)[0] != _lib.DSRG_E_INTRUDER
    q = make_problem(2, 0, 3, 6, seed=1, s=float("inf"))
    q.eps[:] = [-1.0, -0.5, 0.25, 0.75, 2.0]
    q.eps[4] = -1.0 - 0.5 - 0.25                  # e0 + e1 - e2 - e4 = 0
    rc, r = _call(q)
    assert rc == _lib.DSRG_E_INTRUDER and r.e2 == 12345.0
    q = make_problem(1, 2, 2, 6, seed=1, s=float("inf"))
    q.eps[3] = q.eps[0]                           # core-virtual singles denominator 0
    assert _call(q)[0] == _lib.DSRG_E_INTRUDER
    q2 = make_problem(1, 2, 2, 6, seed=1, s=0.5)
    q2.eps[3] = q2.eps[0]
    assert _call(q2)[0] != _lib.DSRG_E_INTRUDER
    # an all-active quadruple carries no amplitude: a zero denominator there is allowed
    q = make_problem(1, 2, 2, 6, seed=1, s=float("inf"))
    q.eps[1] = q.eps[2] = 0.0
    assert _call(q)[0] != _lib.DSRG_E_INTRUDER


def test_workspace_and_batch_checks(lib):
    """workspace_cap below one (PP|PP) batch row, or a virt_batch that does not fit it:
    DSRG_E_OOM before any device work; negative virt_batch: DSRG_E_ARG."""
    p = make_problem(1, 2, 6, 6, seed=1)
    nP = 8
    kp = nP * (nP - 1) // 2
    row = 8 * (nP ** 3 + nP * (2 * kp + nP))
    rc, r = _call(p, opt=_opt(cap=row - 8))
    assert rc == _lib.DSRG_E_OOM and r.e2 == 12345.0
    assert "below one" in lib.dsrg_last_error().decode()
    rc, _ = _call(p, opt=_opt(cap=3 * row, virt_batch=4))
    assert rc == _lib.DSRG_E_OOM
    rc, _ = _call(p, opt=_opt(virt_batch=-1))
    assert rc == _lib.DSRG_E_ARG


def test_nonfinite_fock_offdiag(lib):
    p = make_problem(1, 2, 3, 6, seed=1, f_sigma=0.1)
    p.f_offdiag[0, 4] = np.nan
    rc, r = _call(p)
    assert rc == _lib.DSRG_E_NONFINITE and r.e2 == 12345.0


def test_struct_layouts_match_header(lib):
    """The binding's structs have the sizes of the C declarations (new fields appended)."""
    assert ctypes.sizeof(_lib.Problem) == 4 * 4 + 5 * 8 + 8 + 8 + 8
    assert ctypes.sizeof(_lib.Options) == 4 + 4 + 8 + 8 + 8
    assert _lib.Result.e_total.offset > _lib.Result.role_bytes.offset


def test_active_rdms_argument_checks(lib):
    ci = np.ones((3, 3)) / 3.0
    assert _lib.load().dsrg_active_rdms(ci.ctypes.data, 0, 0, 0, None, None, None, None) == _lib.DSRG_E_UNSUPPORTED
    assert _lib.load().dsrg_active_rdms(ci.ctypes.data, 17, 1, 1, None, None, None, None) == _lib.DSRG_E_UNSUPPORTED
    g1, g2 = np.zeros(2 * 9), np.zeros(3 * 81)
    assert _lib.load().dsrg_active_rdms(ci.ctypes.data, 3, 4, 1, None, g1.ctypes.data, g2.ctypes.data,
                                        None) == _lib.DSRG_E_ARG
    assert _lib.load().dsrg_active_rdms(None, 3, 1, 1, None, g1.ctypes.data, g2.ctypes.data,
                                        None) == _lib.DSRG_E_ARG


def test_relaxed_argument_checks(lib):
    """dsrg_pt3_energy_relaxed: electron numbers outside [0, nA] (DSRG_E_ARG), densities of
    another electron count (DSRG_E_RDM), a non-finite start vector (DSRG_E_NONFINITE) and
    null results (DSRG_E_ARG) are rejected before any device work."""
    assert ctypes.sizeof(_lib.RelaxedResult) == 4 * 8 + 4 * 4
    assert ctypes.sizeof(_lib.RelaxedOutputs) == 4 * 8
    p = make_problem(1, 3, 2, 6, seed=1)
    keep = []
    st, fl = _lib._problem_struct(p, keep)
    r, x, o = _lib.Result(), _lib.RelaxedResult(), _lib.RelaxedOutputs()
    f = lib.dsrg_pt3_energy_relaxed
    opt = ctypes.byref(_lib._options(fl))
    assert f(ctypes.byref(st), 4, 1, None, opt, ctypes.byref(r), ctypes.byref(x), ctypes.byref(o)) == _lib.DSRG_E_ARG
    assert f(ctypes.byref(st), -1, 1, None, opt, ctypes.byref(r), ctypes.byref(x), ctypes.byref(o)) == _lib.DSRG_E_ARG
    assert f(ctypes.byref(st), p.n_alpha, p.n_beta, None, opt, ctypes.byref(r), None, None) == _lib.DSRG_E_ARG
    # make_problem(nA = 3) has 2 alpha and 1 beta electrons
    assert (p.n_alpha, p.n_beta) == (2, 1)
    assert f(ctypes.byref(st), 1, 2, None, opt, ctypes.byref(r), ctypes.byref(x), ctypes.byref(o)) == _lib.DSRG_E_RDM
    bad = np.array(p.ci, dtype=np.float64)
    bad[0, 0] = np.nan
    assert f(ctypes.byref(st), 2, 1, bad.ctypes.data, opt, ctypes.byref(r), ctypes.byref(x),
             ctypes.byref(o)) == _lib.DSRG_E_NONFINITE


def test_dyall_argument_checks(lib):
    """dsrg_dyall_aavv: null outputs (DSRG_E_ARG), active spaces outside 1..9
    (DSRG_E_UNSUPPORTED), and the problem checks of the energy entry points (negative sizes,
    non-finite integrals) before any device work."""
    p = make_problem(1, 3, 2, 6, seed=1)
    keep = []
    st, fl = _lib._problem_struct(p, keep)
    f = lib.dsrg_dyall_aavv
    opt = ctypes.byref(_lib._options(fl))
    t = np.full(3 * 2 * 2 * 3 * 3, 7.0)
    assert f(ctypes.byref(st), opt, None, None) == _lib.DSRG_E_ARG
    assert f(None, opt, t.ctypes.data, None) == _lib.DSRG_E_ARG
    for nA in (0, 10):
        q = make_problem(0, nA, 1, 4, seed=2, with_gamma3=False)
        sq, _ = _lib._problem_struct(q, keep)
        assert f(ctypes.byref(sq), opt, t.ctypes.data, None) == _lib.DSRG_E_UNSUPPORTED
    st.n_virtual = -1
    assert f(ctypes.byref(st), opt, t.ctypes.data, None) == _lib.DSRG_E_ARG
    st.n_virtual = 2
    bad = np.array(p.B)
    bad[0, 0, 0] = np.inf
    st.B = bad.ctypes.data
    assert f(ctypes.byref(st), opt, t.ctypes.data, None) == _lib.DSRG_E_NONFINITE
    assert np.all(t == 7.0)


def test_tile_rules_argument_checks(lib):
    """dsrg_set_tile_rules validates and replaces the rule table without device work."""
    R = _lib.TileRule
    assert ctypes.sizeof(R) == 16
    arr = (R * 2)(R(0, 100, 128, 0), R(101, 200, 0, 8))
    assert lib.dsrg_set_tile_rules(arr, 2) == 0
    assert lib.dsrg_set_tile_rules(arr, -1) == _lib.DSRG_E_ARG
    assert lib.dsrg_set_tile_rules(None, 1) == _lib.DSRG_E_ARG
    bad = (R * 1)(R(50, 10, 0, 0))
    assert lib.dsrg_set_tile_rules(bad, 1) == _lib.DSRG_E_ARG
    bad = (R * 1)(R(0, 10, -1, 0))
    assert lib.dsrg_set_tile_rules(bad, 1) == _lib.DSRG_E_ARG
    assert lib.dsrg_set_tile_rules(None, 0) == 0
