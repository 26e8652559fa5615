"""CPU oracle for the Monte-Carlo shot pipeline (test infrastructure only).

This package is a plain, slow, obviously-correct CPU reference of what the
GPU path computes: code construction, circuit generation, counter-based noise,
Pauli-frame sampling, a stabilizer tableau, detector-error-model extraction by
single-fault injection, min-sum belief propagation (FP64 reference and FP32
decision precision), OSD-0, exhaustive maximum-likelihood decoding and the
logical-error-rate statistic.  Floating point is FP64 unless the function says
otherwise.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
this package never imports the product library.  The two share no code: the
only common module is ``workloads`` (circuit specifications and seeds, which
hold none of the method's arithmetic).

Parity status of each module is stated in its own header.
"""
