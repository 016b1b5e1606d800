"""FP64 CPU oracle for the spin-1 split-step Fourier method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code, table or
helper with the HIP library; the only things both sides see are seeded input
arrays from ``tests/inputs.py`` (which holds none of the method's arithmetic)
and the published definition of the Philox4x64-10 counter generator, which
each side implements on its own.

Modules
-------
philox  -- Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the
           52-bit uniform / Box-Muller draw used for the Wigner noise.
fft     -- an own iterative radix-2 FFT along one axis and an O(N^2) DFT.
spin1   -- the method: grid, Wigner initial state, exact local update,
           kinetic + quadratic-Zeeman step, Strang step, observables,
           transverse-spin structure factor, and the paper's literal
           Lie-order scheme (Eqs. (3)-(5)) for cross-checks.

Every function states which part of the paper (arXiv:2310.03636,
"Universal Dynamics at the Lowest Temperatures") it follows.
"""
