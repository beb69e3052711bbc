"""FP64 CPU oracle for the MALI / FAS / FMG non-LTE radiative-transfer method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this package.
The product path (the HIP library and its Python binding) never does.

This is a plain, slow, deliberately unoptimised restatement of the method of
Bjørgen & Leenaarts (2017), "Numerical non-LTE 3D radiative transfer using a
multigrid method", in FP64 NumPy/SciPy:

* ``physics``   local physics fixed by the atmosphere (Sect. 2.1: collisions and
                background are constant and set by the input atmosphere).
* ``angles``    the 24-direction A4 quadrature (Sect. 3).
* ``levels``    grid hierarchy and coarse atmospheres (Sect. 4.1, 4.2, 4.7).
* ``formal``    short-characteristics formal solution with accumulation of the
                preconditioned mean intensity and the diagonal operator (Eq. 1,
                Sect. 3).
* ``rates``     rate matrix, particle conservation closure and the operator W
                (Eqs. 2-5).
* ``transfer``  full-weighting restriction and trilinear prolongation (Sect. 4.4,
                4.5).
* ``solver``    MALI iteration, FAS V-cycle and full multigrid with the relative
                correction and negative-population repair (Sect. 2.2, 2.3, 4.6,
                4.10, 4.11, 4.12; Eqs. 6-14, 16-18, 21).

The oracle shares no code with the HIP path; only the seeded input generators in
``paper_1701_01607_amd.synth`` feed both, and the oracle does not import them.

Parity unpinned: exact six-level populations on random 3D atmospheres have no
external truth; they are pinned only through the invariants and special cases
that exercise the same code (see tests/test_oracle_*.py).
"""
