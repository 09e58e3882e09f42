"""GPU parity for active spaces of 9 to 16 orbitals: the three-body cumulant over
(2 nA)^6 spin-orbital elements, its energy terms (Sec. III, Eq. E_cumulant: O(N_A^6 N_V)),
the density expansion with more than 256 lower tuples per row and the singles kernel with
more than 64 active terms per element.  Reference values are the FP64 oracle's, stored by
tests/golden/make_golden.py big-active (the dense engine up to 10 active orbitals, the
block-sparse level beyond); compared at 1e-10 relative like the other parity tests."""
import json
import os
import sys

import numpy as np
import pytest

from paper_1701_02011_amd import _lib
from paper_1701_02011_amd.synth import make_problem, random_ci

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "big_active.json")


def _cases():
    with open(GOLDEN) as f:
        return json.load(f)["cases"]


def _close(x, ref, rel=1e-10):
    return abs(x - ref) <= rel * max(1.0, abs(ref))


@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_big_active_against_oracle(case):
    p = make_problem(**case["args"])
    print("big active", case["name"], case["args"], flush=True)
    sys.stdout.flush()
    g = _lib.dsrg_pt3_energy(p)
    for k in ("e2", "e3_a", "e3_b"):
        assert _close(g[k], case[k]), (k, g[k], case[k])


def test_cas12_densities_from_the_gpu():
    """CAS(12,12) (853 776 determinants) end to end on the GPU: the densities of the CAS
    vector from dsrg_active_rdms feed the energy; the energies equal those from the input
    generator's densities (the same expectation values built on the host)."""
    p = make_problem(2, 12, 6, 24, seed=95)
    print("cas12 gpu densities", flush=True)
    sys.stdout.flush()
    g1, g2, g3 = _lib.dsrg_active_rdms(p.ci, 12, p.n_alpha, p.n_beta)
    for a, b in zip((g1, g2, g3), (p.gamma1, p.gamma2, p.gamma3)):
        assert np.abs(np.asarray(a) - b).max() < 1e-13
    import dataclasses
    q = dataclasses.replace(p, gamma1=np.asarray(g1), gamma2=np.asarray(g2), gamma3=np.asarray(g3))
    ref = _lib.dsrg_pt3_energy(p)
    got = _lib.dsrg_pt3_energy(q)
    for k in ("e2", "e3"):
        assert _close(got[k], ref[k], 1e-12), (k, got[k], ref[k])
