"""FP64 CPU oracle for the signature-kernel schemes.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or run anything in this
package.  The GPU library (``paper_2502_08470_amd``) shares no code, table or
helper with it, and never falls back to it.

* ``oracle.schemes`` -- numpy, literal, slow; follows the paper's definitions
  including general time partitions.  Used on small inputs and to pin the C
  oracle.
* ``oracle.c_oracle`` -- ctypes binding of ``sko.c`` (plain C, FP64, OpenMP
  over pairs, exponent tracking) for parity checks at realistic sizes.
* ``oracle.derivatives`` -- gradients of the oracle's forward maps (complex
  step and central finite differences).

Parity status of every function is stated in its module docstring.
"""
