"""CPU oracle for low-precision normalized IHT (QIHT), Guerel et al., IEEE TSP 68 (2020).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain, FP64 reference
that the HIP path is checked against.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  The product path (``paper_1802_04907_amd``) never imports,
links or executes anything in here, and the two share no code.

Modules
-------
philox     Philox4x32-10 counter-based generator (Salmon et al., SC'11).
quantizer  Stochastic quantizer Q(v, b) of Sec. III-A (max-abs scaled,
           unbiased randomized rounding to equispaced levels in [-1, 1]).
niht       Hard threshold H_s, the normalized step size (Eq. step_size),
           the backtracking rule, Algorithm 1 (NIHT) and Algorithm 2 (QIHT),
           and the least-squares refit on the recovered support.
lowprec    Deterministic BF16 / FP8-E4M3 storage of Phi with power-of-two
           row scales (the shared-Phi variant; not in the paper).
complex_niht  Algorithm 2 with a complex unknown x, in complex128
           arithmetic (conjugate-transpose gradient, H_s by modulus).

Every function is pinned by ``tests/test_oracle_*.py`` against something
other than itself (rocRAND's Philox, closed forms, brute force, invariants
stated in the paper).
"""

from . import philox, quantizer, niht, lowprec, complex_niht  # noqa: F401
