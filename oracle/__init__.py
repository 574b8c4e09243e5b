"""Oracle for the batched linear-ODE least-squares solve (TEST INFRASTRUCTURE).

Plain, slow, obviously-correct CPU implementations of what the solve computes,
written from the paper (Scalable Mechanistic Neural Networks, Sec. 3.1,
Eqs. 4-9, and Appendix A.1-A.3).  Only the tests, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import anything in here; the
product library never does, and shares no code with it.

Modules
  dense   -- the definition: dense weighted constraint matrix (App. A.1) and
             its least-squares minimiser by Householder QR (LAPACK), the
             normal-matrix blocks of App. A.2, the adjoint of Eq. 14, the
             per-row closed-form parameter gradients, and (for pinning) torch
             float64 autograd through the dense QR solve.
  banded  -- the same least-squares problem solved by a sequential Householder
             QR over the time-ordered rows (plain C, ``banded.c``), for
             sequences too long for the dense matrix.  Same result up to
             rounding order; cross-pinned against ``dense``.

Parity status of every function is listed in each module's header.
"""
