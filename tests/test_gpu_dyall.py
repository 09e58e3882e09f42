"""GPU parity of the active-to-virtual doubles under Dyall's zeroth-order Hamiltonian
(App. B, Eq. t2_aavv): dsrg_dyall_aavv against the oracle's block-by-block dense solves
(oracle/dyall.py), element by element, and the smallest shifted denominator."""
import sys

import numpy as np
import pytest

from paper_1701_02011_amd import _lib
from paper_1701_02011_amd.synth import make_problem, make_config
from oracle import dyall
from oracle.spaces import Spaces, so_energies

pytestmark = pytest.mark.gpu


def _blocks(t, nA, nV):
    """Oracle spin-orbital t[e, f, u, v] (virtual, active; alpha then beta) -> aa, ab, bb."""
    a, b = slice(0, nA), slice(nA, 2 * nA)
    va, vb = slice(0, nV), slice(nV, 2 * nV)
    return np.stack([t[va, va, a, a], t[va, vb, a, b], t[vb, vb, b, b]])


def _oracle_dmin(p, K, d):
    sp = Spaces(p.n_core, p.n_active, p.n_virtual)
    eps = so_energies(sp, p.eps)
    ev = eps[sp.V]
    D = dyall.shifted_denominators(K, d, ev)
    _, spin = sp.so_index()
    sv, sa = spin[sp.V], spin[sp.A]
    iu, iv = np.triu_indices(2 * sp.nA, k=1)
    nv2 = 2 * sp.nV
    e_lt_f = np.triu(np.ones((nv2, nv2), bool), k=1)[:, :, None]
    allowed = (sv[:, None, None] + sv[None, :, None]) == (sa[iu] + sa[iv])[None, None, :]
    m = e_lt_f & allowed
    return float(np.abs(D[m]).min()) if m.any() else float("inf")


@pytest.mark.parametrize("shape,seed", [((1, 3, 2, 6), 31), ((0, 2, 3, 8), 32), ((1, 1, 3, 6), 33),
                                        ((0, 9, 2, 6), 34), ((2, 4, 5, 12), 35)])
def test_dyall_micro_against_oracle(shape, seed):
    p = make_problem(*shape, seed=seed)
    print("dyall", shape, seed, flush=True)
    sys.stdout.flush()
    t_ref, K, d = dyall.solve(p)
    ref = _blocks(t_ref, p.n_active, p.n_virtual)
    t, dmin = _lib.dsrg_dyall_aavv(p)
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(t - ref).max() <= 1e-10 * scale
    dref = _oracle_dmin(p, K, d)
    assert abs(dmin - dref) <= 1e-12 * max(1.0, abs(dref))


@pytest.mark.parametrize("name", ["tiny", "small"])
def test_dyall_workloads_against_oracle(name):
    p = make_config(name)
    print("dyall", name, flush=True)
    sys.stdout.flush()
    t_ref, K, d = dyall.solve(p)
    ref = _blocks(t_ref, p.n_active, p.n_virtual)
    t, dmin = _lib.dsrg_dyall_aavv(p)
    err = np.abs(t - ref).max()
    assert err <= 1e-10 * max(1.0, np.abs(ref).max()), err
    dref = _oracle_dmin(p, K, d)
    assert abs(dmin - dref) <= 1e-12 * max(1.0, abs(dref))


def test_dyall_device_pointers_and_unsupported():
    import torch
    p = make_problem(1, 3, 4, 9, seed=36)
    t_host, dmin_host = _lib.dsrg_dyall_aavv(p)
    dev = _lib.to_device(p)
    keep = []
    st, fl = _lib._problem_struct(dev, keep)
    tt = torch.zeros((3, 4, 4, 3, 3), dtype=torch.float64, device="cuda:0")
    dm = torch.zeros(1, dtype=torch.float64, device="cuda:0")
    rc = _lib.load().dsrg_dyall_aavv(_lib.ctypes.byref(st), _lib.ctypes.byref(_lib._options(fl)),
                                     tt.data_ptr(), dm.data_ptr())
    assert rc == 0
    assert np.array_equal(tt.cpu().numpy(), t_host)
    assert dm.item() == dmin_host
    q = make_problem(0, 10, 1, 4, seed=37, with_gamma3=False)
    with pytest.raises(_lib.DsrgError) as ei:
        _lib.dsrg_dyall_aavv(q)
    assert ei.value.code == _lib.DSRG_E_UNSUPPORTED
