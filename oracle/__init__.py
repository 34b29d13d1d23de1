"""CPU oracle for the Ozaki-Bailey FFT -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously-correct reference that the GPU
path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or execute anything here; the
product library never does, and it shares no code, header, table or constant
generator with this package.

Modules
-------
constants   number-theoretic constants of the modulus sets (Sec. 2, Eq. capacity;
            Sec. 4.2, Eqs. fcrt and slicing; Sec. 5.1 fractional lift)
roots       quantised roots of unity and double-double twiddles (mpmath)
crt_ref     big-integer Phase A / Kulisch / lift / pack reference (Sec. 4.2,
            Sec. 5.1, Alg. 2)
exact       ctypes front end of ``exact.c`` (the exact-pipeline transform) and
            ``dd.c`` (the double-double DFT)
"""
