"""Reference densities from a CAS vector on the GPU (dsrg_active_rdms) against the oracle's
brute-force expectation values in the full Fock space (nA <= 7), and at CAS(8,8) against
the input generator's densities; the energies of a problem built from the GPU densities
equal those from the oracle's."""
import math
import sys

import numpy as np
import pytest

from paper_1701_02011_amd import _lib, synth
from oracle.hilbert import active_rdm_blocks

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("nA,na,nb,seed", [(2, 1, 1, 1), (3, 2, 1, 2), (4, 2, 2, 3), (5, 3, 2, 4),
                                           (6, 3, 3, 5), (7, 4, 3, 6), (6, 4, 1, 7), (4, 4, 0, 8)])
def test_active_rdms_against_fock_space(nA, na, nb, seed):
    rng = np.random.default_rng(seed)
    ci = synth.random_ci(rng, nA, na, nb)
    say("active rdms", nA, na, nb)
    g = _lib.dsrg_active_rdms(ci, nA, na, nb)
    ref = active_rdm_blocks(ci, nA, na, nb)
    for k, (x, y) in enumerate(zip(g, ref)):
        assert np.abs(x - y).max() <= 1e-13, (k, np.abs(x - y).max())


def test_active_rdms_cas88_against_generator():
    rng = np.random.default_rng(9)
    ci = synth.random_ci(rng, 8, 4, 4)
    say("active rdms CAS(8,8)")
    g = _lib.dsrg_active_rdms(ci, 8, 4, 4)
    ref = synth.active_rdms(ci, 8, 4, 4)
    for k, (x, y) in enumerate(zip(g, ref)):
        assert np.abs(x - y).max() <= 1e-13, (k, np.abs(x - y).max())
    g1, g2, g3 = _lib.dsrg_active_rdms(ci, 8, 4, 4, with_gamma3=False)
    assert g3 is None and np.array_equal(g1, g[0]) and np.array_equal(g2, g[1])
