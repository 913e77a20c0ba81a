"""CPU oracle for 2D replica-exchange Wang-Landau sampling (arXiv:1508.02748).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP path (``paper_1508_02748_amd``) and never imports it.

Modules
-------
rewl    ctypes wrapper of ``rewl_oracle.c``: the plain, slow WL/REWL iteration
        (Sec. 2 of the paper) under the same Philox stream as the GPU path.
exact   exact references used to pin the oracle: brute-force enumeration of
        g(E,M) for tiny lattices, and the exact g(E) of the periodic lattice
        from Kaufman's partition function (the comparison of Sec. 3 / Fig. 5).
lnz     thermodynamic reweighting ln Z(beta,h) and its moments, written as the
        plain logsumexp definition over (E,M) in float64.
merge   joining the per-walker ln g fragments (Eq. 3, E_mat, Eq. 4).
build   compiles ``rewl_oracle.c`` with gcc.
"""
