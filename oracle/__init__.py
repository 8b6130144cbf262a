"""CPU oracle for the multi-component progressive codec (TEST INFRASTRUCTURE).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library under
``paper_2308_11759_amd``) never imports it and shares no code with it.

Layout:
  pmc_oracle.c   plain serial C block codec (format version 1), built with
                 ``gcc -O2 -ffp-contract=off`` into ``liboracle.so``
  driver.py      Alg. 1 (multi-component compression) and Alg. 2 (progressive
                 reconstruction) of the paper (Sec. 4.1, 4.2) over any codec
"""
from .lib import load, build  # noqa: F401
