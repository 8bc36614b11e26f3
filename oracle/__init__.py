"""ORACLE -- test infrastructure only.

A plain CPU implementation of what the GPU library computes, written from the
paper's problem statement (Section 2, equation (1)): the value and the full
Jacobian of a sparse polynomial system, term by term, in complex
double-double (``ddoracle``, plain C built with gcc) and in exact Gaussian
rationals (``exact``).  It shares no code with the GPU path and the GPU path
never imports it.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU
baseline of ``bench.py`` may use it.
"""
