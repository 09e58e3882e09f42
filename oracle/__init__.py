"""FP64 CPU oracle for the DSRG-MRPT3 hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link or
execute anything in this package; only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
path: the only module both sides use is the seeded input generator
(``paper_1701_02011_amd.synth``), which holds none of the method's arithmetic.

Layout
------
``spaces``   spin-orbital index spaces, densities and cumulants (step a0).
``gno``      a generic commutator engine for operators normal ordered with respect
             to a multideterminantal reference (Mukherjee-Kutzelnigg generalised
             normal ordering, Sec. II.A).  It converts each normal-ordered operator
             to true-vacuum order with the reference densities, takes the exact
             commutator with the canonical anticommutation relations only, and
             converts back, keeping the scalar, one- and two-body parts (the
             "1,2" truncation, Sec. II.A).  No hand-derived term list is used.
``dsrg``     the DSRG-MRPT3 steps in the paper's order (Sec. II.B):
             first-order amplitudes, E^(2), [H~(1), A(1)]_{1,2}, second-order
             amplitudes, H~(2)_{1,2} and E^(3).
``hilbert``  brute force in the full determinant (Fock) space for micro inputs;
             it pins the engine, the densities and the perturbation limits.

Every floating-point quantity is FP64.  Orbital energies, integrals and densities
come from the caller (the paper poses the method on semicanonical orbitals, DF
integrals and reference cumulants).  Parity status of each function is stated in
its docstring; the values printed in the paper's tables need molecules and are
"parity unpinned".
"""
