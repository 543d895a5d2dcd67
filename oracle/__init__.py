"""CPU oracle for constant-weight PIR over textbook FV.

TEST INFRASTRUCTURE ONLY: the plain, slow reference the GPU library is checked against.  Only the
test suite, the package smoke check and the benchmark's CPU-baseline leg may import it; the
product path never does.  It shares no code with the GPU library.

Parts: `core` (C++ FV and PIR answer through ctypes), `mapping` (Algorithms 3, 7, 8 and the code
length rule), `client` (keys, database and encrypted query from the seeded generators), `micro`
(an independent pure-Python FV for tiny ring degrees).
"""
from .core import Oracle, divmod_big, negacyclic_mul_ntt, negacyclic_mul_schoolbook  # noqa: F401
from .mapping import (binom, code_length, inverse_perfect_map, lossy_map, perfect_map,  # noqa: F401
                      codeword_bits)
