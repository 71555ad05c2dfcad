"""CPU oracle for the BN254-Fr NTT.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call, link or execute
anything in this package. The library under test never does, and the two
share no code: the only common dependency is the seeded input generator in
``seeded_inputs.py``, which holds none of the transform's arithmetic.

* ``fr_ntt``  -- Python big-integer definition (O(N^2)) and textbook radix-2 FFT.
* ``cref``    -- ctypes front end for ``ntt_ref.c`` (plain C, OpenMP), used
                 for sizes the Python oracle cannot reach in seconds.
"""
